// Split-bf16 instantiations of the implicit-GEMM conv (kernel in k_conv_mfma.h):
// float activations, each operand taken as bf16 hi + lo parts on the matrix cores.
#include "k_conv_mfma.h"
#include "k_conv_split64.h"

namespace idq {
namespace mfma {

namespace {

template <int CI, int CO>
int by_epi(const ConvArgs& a, hipStream_t s) {
  if constexpr (CI == 64 && CO <= 4) {
    // image-facing outputs: channel-half pipelined kernel, else the generic one
    if (halves_fits(a)) {
      switch (a.epi) {
        case E_RES: return launch_halves<PREC_SPLIT, CO, E_RES>(a, s);
        case E_SUB: return launch_halves<PREC_SPLIT, CO, E_SUB>(a, s);
        default: return fail(IDQ_E_UNSUPPORTED, "no split-bf16 MFMA epilogue of this kind");
      }
    }
    switch (a.epi) {
      case E_RES: return launch_shape<PREC_SPLIT, CI, CO, P_NONE, E_RES>(a, s);
      case E_SUB: return launch_shape<PREC_SPLIT, CI, CO, P_NONE, E_SUB>(a, s);
      default: return fail(IDQ_E_UNSUPPORTED, "no split-bf16 MFMA epilogue of this kind");
    }
  } else if constexpr (CI == 64) {
    // channel-half pipelined kernel (k_conv_split64.h)
    if (halves_fits(a)) {
      switch (a.epi) {
        case E_ACT: return launch_halves<PREC_SPLIT, CO, E_ACT>(a, s);
        case E_DELTA: return launch_halves<PREC_SPLIT, CO, E_DELTA>(a, s);
        case E_RAW: return launch_halves<PREC_SPLIT, CO, E_RAW>(a, s);
        default: return fail(IDQ_E_UNSUPPORTED, "no split-bf16 MFMA epilogue of this kind");
      }
    }
  }
  if constexpr (CO > 4) {
    switch (a.epi) {
      case E_ACT: return launch_shape<PREC_SPLIT, CI, CO, P_NONE, E_ACT>(a, s);
      case E_DELTA: return launch_shape<PREC_SPLIT, CI, CO, P_NONE, E_DELTA>(a, s);
      case E_RAW: return launch_shape<PREC_SPLIT, CI, CO, P_NONE, E_RAW>(a, s);
      default: return fail(IDQ_E_UNSUPPORTED, "no split-bf16 MFMA epilogue of this kind");
    }
  }
}

}  // namespace

int launch_split(const ConvArgs& a, hipStream_t s) {
  if (a.pro != P_NONE) return fail(IDQ_E_UNSUPPORTED, "split passes take plain operands");
#define X(A, B) \
  if (a.CI == A && a.CO == B) return by_epi<A, B>(a, s);
  IDQ_MFMA_SPLIT(X)
#undef X
  return fail(IDQ_E_UNSUPPORTED, "no split-bf16 MFMA instantiation for this shape");
}

}  // namespace mfma
}  // namespace idq
