// f32 instantiations of the implicit-GEMM conv (kernel in k_conv_mfma.h; plain
// passes from 64 channels in the channel-half pipelined kernel, k_conv_split64.h).
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
        case E_ACT: return launch_halves<PREC_F32, CO, E_ACT>(a, s);
        case E_DELTA: return launch_halves<PREC_F32, CO, E_DELTA>(a, s);
        case E_RAW: return launch_halves<PREC_F32, CO, E_RAW>(a, s);
        default: break;  // E_DDOT: the generic kernel
      }
    }
  }
  switch (a.epi) {
    case E_ACT: return launch_shape<PREC_F32, CI, CO, PRO, E_ACT>(a, s);
    case E_DELTA: return launch_shape<PREC_F32, CI, CO, PRO, E_DELTA>(a, s);
    case E_RAW: return launch_shape<PREC_F32, CI, CO, PRO, E_RAW>(a, s);
    case E_DDOT: return launch_shape<PREC_F32, CI, CO, PRO, E_DDOT>(a, s);
    default: return fail(IDQ_E_UNSUPPORTED, "no fp32 MFMA epilogue of this kind");
  }
}

template <int CI, int CO>
int thin(const ConvArgs& a, hipStream_t s) {
  const bool jvp = a.pro == P_JVP;
  if (a.epi == E_RES && !jvp) return launch_shape<PREC_F32, CI, CO, P_NONE, E_RES>(a, s);
  if (a.epi == E_ADD && !jvp) return launch_shape<PREC_F32, CI, CO, P_NONE, E_ADD>(a, s);
  if (a.epi == E_SUB) {
    if (jvp) return launch_shape<PREC_F32, CI, CO, P_JVP, E_SUB>(a, s);
    return launch_shape<PREC_F32, CI, CO, P_NONE, E_SUB>(a, s);
  }
  return fail(IDQ_E_UNSUPPORTED, "no fp32 MFMA epilogue of this kind");
}

}  // namespace

int launch_f32(const ConvArgs& a, hipStream_t s) {
  const bool jvp = a.pro == P_JVP;
#define X(A, B)                                                                        \
  if (a.CI == A && a.CO == B) {                                                        \
    if (jvp) {                                                                         \
      if (A <= 4 || a.epi != E_RAW)                                                    \
        return fail(IDQ_E_UNSUPPORTED, "tangent prologue: wide operand, raw output");  \
      return launch_shape<PREC_F32, A, B, (A > 4 ? P_JVP : P_NONE), E_RAW>(a, s);      \
    }                                                                                  \
    return by_epi<A, B, P_NONE>(a, s);                                                 \
  }
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
