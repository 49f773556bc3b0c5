// bf16 instantiations of the implicit-GEMM conv (kernel in k_conv_mfma.h).
#include "k_conv_mfma.h"
#include "k_conv_split64.h"

namespace idq {
namespace mfma {

namespace {

template <int CI, int CO, int PRO>
int by_epi(const ConvArgs& a, hipStream_t s) {
  if constexpr (CI == 64 && (CO == 64 || CO == 32) && PRO == P_NONE) {
    if (halves_fits(a)) {
      switch (a.epi) {
        case E_ACT: return launch_halves<PREC_BF16, CO, E_ACT>(a, s);
        case E_DELTA: return launch_halves<PREC_BF16, CO, E_DELTA>(a, s);
        case E_RAW: return launch_halves<PREC_BF16, CO, E_RAW>(a, s);
        default: break;
      }
    }
  }
  switch (a.epi) {
    case E_ACT: return launch_shape<PREC_BF16, CI, CO, PRO, E_ACT>(a, s);
    case E_DELTA: return launch_shape<PREC_BF16, CI, CO, PRO, E_DELTA>(a, s);
    case E_RAW: return launch_shape<PREC_BF16, CI, CO, PRO, E_RAW>(a, s);
    default: return fail(IDQ_E_UNSUPPORTED, "no bf16 MFMA epilogue of this kind");
  }
}

template <int CI, int CO>
int thin(const ConvArgs& a, hipStream_t s) {
  if (a.epi == E_RES) return launch_shape<PREC_BF16, CI, CO, P_NONE, E_RES>(a, s);
  if (a.epi == E_ADD) return launch_shape<PREC_BF16, CI, CO, P_NONE, E_ADD>(a, s);
  if (a.epi == E_SUB) return launch_shape<PREC_BF16, CI, CO, P_NONE, E_SUB>(a, s);
  return fail(IDQ_E_UNSUPPORTED, "no bf16 MFMA epilogue of this kind");
}

}  // namespace

int launch_bf16(const ConvArgs& a, hipStream_t s) {
  if (a.pro != P_NONE) return fail(IDQ_E_UNSUPPORTED, "bf16 passes take plain operands");
#define X(A, B) \
  if (a.CI == A && a.CO == B) return by_epi<A, B, P_NONE>(a, s);
  IDQ_MFMA_WIDE(X)
#undef X
#define X(A, B) \
  if (a.CI == A && a.CO == B) return thin<A, B>(a, s);
  IDQ_MFMA_THIN(X)
#undef X
  return fail(IDQ_E_UNSUPPORTED, "no MFMA instantiation for this shape");
}

}  // namespace mfma
}  // namespace idq
