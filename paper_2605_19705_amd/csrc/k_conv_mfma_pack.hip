// Shape table and weight packing of the implicit-GEMM conv (k_conv_mfma.h).
#include "k_conv_mfma.h"

namespace idq {

namespace mfma {
int launch_bf16(const ConvArgs& a, hipStream_t s);  // k_conv_mfma_bf16.hip
int launch_f32(const ConvArgs& a, hipStream_t s);   // k_conv_mfma_f32.hip
int launch_split(const ConvArgs& a, hipStream_t s); // k_conv_mfma_split.hip
}  // namespace mfma

bool mfma_supported(int prec, int ci, int co) {
  if (prec == PREC_SPLIT) {
#define X(A, B) if (ci == A && co == B) return true;
    IDQ_MFMA_SPLIT(X)
#undef X
    return false;
  }
  if (prec != PREC_BF16 && prec != PREC_F32) return false;
#define X(A, B) if (ci == A && co == B) return true;
  IDQ_MFMA_WIDE(X)
  IDQ_MFMA_THIN(X)
#undef X
  return false;
}

// Weights in fragment order: [chunk][co block j][lane][16 bytes], the lane's
// slice being co = 16 j + lane % 16 and k = chunk * KC + (lane / 16) * V + e.
// Split: the bf16 hi parts in that order, followed by the bf16-rounded
// remainders w - hi in the same order.
size_t pack_mfma_weights(int prec, int ci, int co, const double* w, void* dst) {
  const bool split = prec == PREC_SPLIT;
  const bool bf = prec == PREC_BF16 || split;
  const int V = bf ? 8 : 4, KC = 4 * V, K = 9 * ci;
  const int nch = (K + KC - 1) / KC, nj = (co + 15) / 16;
  const size_t one = static_cast<size_t>(nch) * nj * 64 * 16;
  const size_t bytes = split ? 2 * one : one;
  if (!dst) return bytes;
  for (int ch = 0; ch < nch; ++ch)
    for (int j = 0; j < nj; ++j)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < V; ++e) {
          const int o = 16 * j + (l % 16);
          const int k = ch * KC + (l / 16) * V + e;
          double v = 0.0;
          if (o < co && k < K) v = w[(static_cast<size_t>(o) * ci + k % ci) * 9 + k / ci];
          const size_t idx = ((static_cast<size_t>(ch) * nj + j) * 64 + l) * V + e;
          if (split) {
            const float f = static_cast<float>(v);
            const bf16 hi = f2bf(f);
            static_cast<bf16*>(dst)[idx] = hi;
            static_cast<bf16*>(dst)[one / 2 + idx] = f2bf(f - bf2f(hi));
          } else if (bf) {
            static_cast<bf16*>(dst)[idx] = f2bf(static_cast<float>(v));
          } else {
            static_cast<float*>(dst)[idx] = static_cast<float>(v);
          }
        }
  return bytes;
}

int launch_conv_mfma(const ConvArgs& a, int prec, hipStream_t s) {
  if (prec == PREC_SPLIT) return mfma::launch_split(a, s);
  return prec == PREC_BF16 ? mfma::launch_bf16(a, s) : mfma::launch_f32(a, s);
}

}  // namespace idq
