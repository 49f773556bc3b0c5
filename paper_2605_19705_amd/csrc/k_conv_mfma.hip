// Implicit-GEMM 3x3 conv on the gfx950 matrix cores (placeholder until the
// MFMA kernels land; every shape falls back to the direct kernel).
#include "kernels.h"

namespace idq {

bool mfma_supported(int, int, int) { return false; }
size_t pack_mfma_weights(int, int, int, const double*, void*) { return 0; }
int launch_conv_mfma(const ConvArgs&, int, hipStream_t) {
  return fail(IDQ_E_UNSUPPORTED, "MFMA conv not available");
}

}  // namespace idq
