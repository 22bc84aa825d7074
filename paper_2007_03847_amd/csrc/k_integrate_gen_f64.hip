// k_integrate_gen_f64.hip -- F64 instantiations of the integrator for general Ito
// disturbances (IntegArgs::sde): every variant, one trajectory per lane or L
// lanes per trajectory, in a translation unit of their own so that the OU
// kernels are compiled exactly as without them.
#include "k_integrate.hpp"
#include "k_variants.hpp"

namespace fmc {

hipError_t launch_integrate_gen_f64(int variant_id, const IntegArgs<double>& a, int64_t n_groups,
                                    hipStream_t st) {
  int id = 0;
#define FMC_X(NG, PM, L, WPB)                                                                \
  if (variant_id == id) {                                                                    \
    if constexpr (L == 1)                                                                   \
      hipLaunchKernelGGL((k_rk4_lane<double, NG, PM, true>), dim3((unsigned)n_groups), dim3(64), 0, \
                         st, a);                                                             \
    else                                                                                     \
      hipLaunchKernelGGL((k_rk4_group_gen<double, NG, PM, L, WPB>), dim3((unsigned)n_groups),   \
                         dim3(64 * WPB), 0, st, a);                                          \
    return hipGetLastError();                                                                \
  }                                                                                          \
  ++id;
  FMC_VARIANTS(FMC_X)
#undef FMC_X
  return hipErrorInvalidValue;
}

}  // namespace fmc
