// k_integrate_f32.hip -- FP32 instantiations of the integrator variants.
#include "k_integrate.hpp"
#include "k_variants.hpp"

namespace fmc {

hipError_t launch_integrate_f32(int variant_id, const IntegArgs<float>& a, int64_t n_groups,
                                hipStream_t st) {
  int id = 0;
#define FMC_X(NG, PM, L, WPB)                                                              \
  if (variant_id == id) {                                                                  \
    if (a.sde) /* general Ito processes: their own instantiations */                      \
      return launch_integrate_gen_f32(variant_id, a, n_groups, st);                      \
    if constexpr (L == 1)                                                                  \
      hipLaunchKernelGGL((k_rk4_lane<float, NG, PM>), dim3((unsigned)n_groups), dim3(64), 0,   \
                         st, a);                                                           \
    else                                                                                   \
      hipLaunchKernelGGL((k_rk4_group<float, NG, PM, L, WPB>), dim3((unsigned)n_groups),       \
                         dim3(64 * WPB), 0, st, a);                                        \
    return hipGetLastError();                                                              \
  }                                                                                        \
  ++id;
  FMC_VARIANTS(FMC_X)
#undef FMC_X
  return hipErrorInvalidValue;
}

}  // namespace fmc
