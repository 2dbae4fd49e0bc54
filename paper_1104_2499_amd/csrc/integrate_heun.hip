// integrate_heun.hip -- the stochastic Heun instances of the single-set integrator kernel.
#include "integrate.hpp"

namespace abp {

void dispatch_integrate_heun(const FwdArgs &a, const Shape &sh, hipStream_t st)
{
    dispatch_integrate<1>(a, sh, st);
}

}  // namespace abp
