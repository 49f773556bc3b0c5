// Zero-padded 3x3 conv passes of the regularizer network N_theta
// (the conv layers inside g(x) = 1/2 ||x - N(x)||^2, eq. GS).
//
// Two kernel families share one argument block (ConvArgs):
//   * conv_direct: one thread per (pixel, 16 output channels), scalar FMA in the
//     math type.  Used for float64 and for shapes the MFMA kernels do not cover.
//   * conv_mfma (k_conv_mfma.hip): implicit GEMM on the gfx950 matrix cores.
//   * conv_thin (k_conv_thin.hip): image-facing outputs (CO <= 3) from NHWC
//     activations, float32 on the vector ALUs.
// Every pass is   acc[co](p) = sum_{ci, tap} W[co][ci][tap] * a[ci](p + off(tap))
// with the operand a produced by the prologue (Pro) and the result consumed by
// the epilogue (Epi); see kernels.h.

#include "kernels.h"

namespace idq {

namespace {

template <typename TM, typename TS, typename TA>
__device__ inline TM load_operand(const ConvArgs& a, int ni, int ci, int yy, int xx) {
  if (a.in_fmt == F_NCHW) {
    size_t idx = ((static_cast<size_t>(ni) * a.CI + ci) * a.H + yy) * a.W + xx;
    return ld<TM>(static_cast<const TS*>(a.in0), idx);
  }
  size_t idx = ((static_cast<size_t>(ni) * a.H + yy) * a.W + xx) * a.CI + ci;
  TM v = ld<TM>(static_cast<const TA*>(a.in0), idx);
  if (a.pro == P_JVP) {
    TM hd = ld<TM>(static_cast<const TA*>(a.in1), idx);
    return (a.act == IDQ_ACT_SOFTPLUS ? dsp_from_a(v) : TM(1)) * hd;
  }
  return v;
}

template <typename TM, typename TS, typename TA, bool RBF>
__global__ __launch_bounds__(256) void conv_direct_kernel(ConvArgs a) {
  const int HW = a.H * a.W;
  const int p = blockIdx.x * 256 + threadIdx.x;
  const int ni = blockIdx.y;
  const int co0 = blockIdx.z * 16;
  if (p >= HW) return;
  if (!gate_open(a.gate, a.gate_mask, ni / a.img_div)) return;
  if (a.work_px && blockIdx.z == 0) atomicAdd(a.work_px, 1ull);
  const int y = p / a.W, x = p - (p / a.W) * a.W;
  const int nco = min(16, a.CO - co0);
  const TM* w = static_cast<const TM*>(a.wgt);
  TM acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = TM(0);
  for (int ci = 0; ci < a.CI; ++ci) {
    for (int t = 0; t < 9; ++t) {
      const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
      if (yy < 0 || yy >= a.H || xx < 0 || xx >= a.W) continue;
      TM v = load_operand<TM, TS, TA>(a, ni, ci, yy, xx);
      if (RBF) v = static_cast<TM>(round_bf(static_cast<float>(v)));
      const TM* wp = w + (static_cast<size_t>(co0) * a.CI + ci) * 9 + t;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (j < nco) acc[j] += wp[static_cast<size_t>(j) * a.CI * 9] * v;
    }
  }
  const TM* bias = static_cast<const TM*>(a.bias);
  const bool sp = a.act == IDQ_ACT_SOFTPLUS;
  for (int j = 0; j < 16; ++j) {
    if (j >= nco) break;
    const int co = co0 + j;
    const TM b = bias ? bias[co] : TM(0);
    if (a.out_fmt == F_NCHW) {
      size_t o = ((static_cast<size_t>(ni) * a.CO + co) * a.H + y) * a.W + x;
      TS* out = static_cast<TS*>(a.out0);
      const TS* e0 = static_cast<const TS*>(a.e0);
      TM r;
      switch (a.epi) {
        case E_ACT: r = sp ? softplus_f(acc[j] + b) : acc[j] + b; break;
        case E_RES: r = ld<TM>(e0, o) - (acc[j] + b); break;
        case E_ADD: r = ld<TM>(e0, o) + (acc[j] + b); break;
        case E_SUB: r = ld<TM>(e0, o) - acc[j]; break;
        default: r = acc[j]; break;
      }
      st(out, o, r);
    } else {
      size_t o = ((static_cast<size_t>(ni) * a.H + y) * a.W + x) * a.CO + co;
      TA* out = static_cast<TA*>(a.out0);
      const TA* e0 = static_cast<const TA*>(a.e0);
      switch (a.epi) {
        case E_ACT: st(out, o, sp ? softplus_f(acc[j] + b) : acc[j] + b); break;
        case E_RAW: st(out, o, acc[j]); break;
        case E_DELTA: {
          TM av = ld<TM>(e0, o);
          st(out, o, (sp ? dsp_from_a(av) : TM(1)) * acc[j]);
          break;
        }
        case E_DDOT: {
          TM av = ld<TM>(e0, o);
          TM hd = ld<TM>(static_cast<const TA*>(a.e1), o);
          TM t = ld<TM>(static_cast<const TA*>(a.e2), o);
          TM s1 = sp ? dsp_from_a(av) : TM(1);
          TM s2 = sp ? s1 * (TM(1) - s1) : TM(0);
          st(out, o, s2 * hd * t + s1 * acc[j]);
          st(static_cast<TA*>(a.out1), o, s1 * t);
          break;
        }
        case E_RES: st(out, o, ld<TM>(e0, o) - (acc[j] + b)); break;
        case E_SUB: st(out, o, ld<TM>(e0, o) - acc[j]); break;
        default: break;
      }
    }
  }
}

}  // namespace

int launch_conv_mfma(const ConvArgs& a, int prec, hipStream_t s);  // k_conv_mfma.hip

// The MFMA kernels read thin (CI <= 4) operands as NCHW state tensors and wide
// ones as NHWC activations, and write NHWC outputs (CO > 4) through E_ACT /
// E_DELTA / E_RAW / E_DDOT (float32) or NCHW outputs (CO <= 4) through E_RES /
// E_SUB; the float32 tangent prologue feeds E_RAW (wide) or E_SUB (thin).
static bool mfma_form_ok(const ConvArgs& a, int prec) {
  // the bf16 kernels evaluate SoftPlus (and its derivative) only
  if (prec == PREC_BF16 && a.act != IDQ_ACT_SOFTPLUS) return false;
  const bool in_ok = a.CI <= 4 ? (a.in_fmt == F_NCHW && a.pro == P_NONE)
                               : (a.in_fmt == F_NHWC && (a.pro == P_NONE || prec == PREC_F32));
  bool out_ok;
  if (a.CO > 4)
    out_ok = a.out_fmt == F_NHWC && (a.epi == E_ACT || a.epi == E_DELTA || a.epi == E_RAW ||
                                     (a.epi == E_DDOT && prec == PREC_F32));
  else
    out_ok = a.out_fmt == F_NCHW && (a.epi == E_RES || a.epi == E_SUB || a.epi == E_ADD) &&
             (a.pro == P_NONE || a.epi == E_SUB);
  const bool jvp_ok = a.pro != P_JVP || (a.CO > 4 ? a.epi == E_RAW : a.epi == E_SUB);
  return in_ok && out_ok && jvp_ok;
}

int launch_conv(const ConvArgs& a, int prec, hipStream_t s) {
  if (a.NI <= 0 || a.H <= 0 || a.W <= 0) return IDQ_OK;
  if (prec == PREC_SPLIT) {
    // no direct-kernel form: callers run shapes without a split kernel as PREC_F32
    if (!a.wmfma || !mfma_supported(prec, a.CI, a.CO) || !mfma_form_ok(a, prec))
      return fail(IDQ_E_UNSUPPORTED, "split-bf16 conv pass of an unsupported form");
    return launch_conv_mfma(a, prec, s);
  }
  if (thin_supported(a, prec)) return launch_conv_thin(a, prec, s);
  if (prec != PREC_F64 && a.wmfma && mfma_supported(prec, a.CI, a.CO) &&
      mfma_form_ok(a, prec))
    return launch_conv_mfma(a, prec, s);
  dim3 grid((a.H * a.W + 255) / 256, a.NI, (a.CO + 15) / 16);
  if (grid.y > 65535) return fail(IDQ_E_INVAL, "too many images in one conv pass");
  if (a.ev0) IDQ_HIP(hipEventRecord(a.ev0, s));
  switch (prec) {
    case PREC_F64:
      conv_direct_kernel<double, double, double, false><<<grid, 256, 0, s>>>(a);
      break;
    case PREC_F32:
      conv_direct_kernel<float, float, float, false><<<grid, 256, 0, s>>>(a);
      break;
    case PREC_BF16:
      conv_direct_kernel<float, float, bf16, true><<<grid, 256, 0, s>>>(a);
      break;
    default:
      return fail(IDQ_E_INVAL, "bad conv precision");
  }
  IDQ_HIP(hipGetLastError());
  if (a.ev1) IDQ_HIP(hipEventRecord(a.ev1, s));
  return IDQ_OK;
}

}  // namespace idq
