// adjoint_em.hip -- the Euler-Maruyama instances of the 16-step adjoint backward kernel for the
// exact gradient. The register-thrifty schedule this file is built with suits them; the 8-step
// and the decayed estimator's instances stay in adjoint.hip, where they measured faster.
#include "adjoint.hpp"

namespace abp {

void launch_backward_em16(int occ, bool zlds, bool subl, unsigned grid, size_t lds,
                          hipStream_t st, const AdjArgs &a)
{
    if (occ == 2)
        launch_backward<0, 0, 16, 2>(zlds, subl, grid, lds, st, a);
    else
        launch_backward<0, 0, 16, 1>(zlds, subl, grid, lds, st, a);
}

}  // namespace abp
