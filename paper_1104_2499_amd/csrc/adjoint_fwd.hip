// adjoint_fwd.hip -- the instances of the adjoint's forward-phase kernel with the noise of the next
// span computed ahead of the steps (the form for ensembles of at most two wavefronts per SIMD).
#include "adjoint.hpp"

namespace abp {

void launch_forward_ahead(bool heun, unsigned grid, hipStream_t st, const AdjArgs &a)
{
    if (heun)
        hipLaunchKernelGGL((k_adj_forward<1, kAhead>), dim3(grid), dim3(256), 0, st, a, a.rows);
    else
        hipLaunchKernelGGL((k_adj_forward<0, kAhead>), dim3(grid), dim3(256), 0, st, a, a.rows);
}

}  // namespace abp
