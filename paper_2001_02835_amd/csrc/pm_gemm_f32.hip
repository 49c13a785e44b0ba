// Instantiations of the interleaved-complex mode-wise product kernel for
// float (FP32 MFMA), one per tile configuration.
#include "pm_gemm_impl.h"

namespace pm {

hipError_t launch_gemm_f32(const GemmArgs& a, int cfg, bool g3, hipStream_t s) {
  switch (cfg) {
#define PM_CASE(I, WM, WN, WGM, WGN) \
  case I:                            \
    return launch_cgemm_cfg<float, WM, WN, WGM, WGN>(a, g3, s);
    PM_GEMM_CONFIGS(PM_CASE)
#undef PM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace pm
