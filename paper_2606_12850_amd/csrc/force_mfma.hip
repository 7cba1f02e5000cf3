// Mixed-precision (BF16/FP16 MFMA) force kernels: not built yet.
#include "semx_internal.hpp"

namespace semx {
bool mfma_supported(int) { return false; }
hipError_t launch_force_mfma(int, int, int, bool, const ForceArgs&, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace semx
