// integrate_em.hip -- the Euler-Maruyama instances of the single-set integrator kernel.
#include "integrate.hpp"

namespace abp {

void dispatch_integrate_em(const FwdArgs &a, const Shape &sh, hipStream_t st)
{
    dispatch_integrate<0>(a, sh, st);
}

}  // namespace abp
