// Zero-padded 3x3 conv passes of the regularizer network N_theta
// (the conv layers inside g(x) = 1/2 ||x - N(x)||^2, eq. GS).
//
// Two kernel families share one argument block (ConvArgs):
//   * conv_direct: one thread per (pixel, 4 output channels) of a 16 x 16 tile,
//     operand halo and weights staged in LDS, scalar FMA in the math type.  Used
//     for float64 and for shapes the MFMA kernels do not cover.
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

// Tile shape of the direct kernel: 16 x 16 output pixels (one per thread) and
// DCO output channels per workgroup; the operand's (18 x 18)-pixel halo is
// staged in LDS DCI input channels at a time, the weights of the workgroup's
// output channels once, so the inner loop reads only LDS (the weights as
// broadcasts).
constexpr int DT = 16, DH = DT + 2, DHP = DH * DH, DCO = 4, DCI = 16;

template <typename TM, typename TS, typename TA, bool RBF>
__global__ __launch_bounds__(256) void conv_direct_kernel(ConvArgs a, int ntx) {
  extern __shared__ __attribute__((aligned(16))) char dsm[];
  TM* halo = reinterpret_cast<TM*>(dsm);             // [DCI][DHP]
  TM* wl = halo + DCI * DHP;                         // [DCO][CI][9]
  const int tid = threadIdx.x;
  const int ni = blockIdx.y;
  const int ty0 = (blockIdx.x / ntx) * DT, tx0 = (blockIdx.x % ntx) * DT;
  const int co0 = blockIdx.z * DCO;
  if (!gate_open(a.gate, a.gate_mask, ni / a.img_div)) return;
  const int ly = tid / DT, lx = tid % DT;
  const int y = ty0 + ly, x = tx0 + lx;
  const bool inside = y < a.H && x < a.W;
  if (a.work_px && blockIdx.z == 0 && inside) atomicAdd(a.work_px, 1ull);
  const int nco = min(DCO, a.CO - co0);
  const TM* w = static_cast<const TM*>(a.wgt);
  for (int i = tid; i < nco * a.CI * 9; i += 256)
    wl[i] = w[static_cast<size_t>(co0) * a.CI * 9 + i];
  TM acc[DCO];
#pragma unroll
  for (int j = 0; j < DCO; ++j) acc[j] = TM(0);
  for (int c0 = 0; c0 < a.CI; c0 += DCI) {
    const int nci = min(DCI, a.CI - c0);
    __syncthreads();  // the previous channel chunk has been read
    for (int i = tid; i < nci * DHP; i += 256) {
      const int cc = i / DHP, hp = i - cc * DHP;
      const int yy = ty0 - 1 + hp / DH, xx = tx0 - 1 + hp % DH;
      TM v = TM(0);
      if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) {
        v = load_operand<TM, TS, TA>(a, ni, c0 + cc, yy, xx);
        if (RBF) v = static_cast<TM>(round_bf(static_cast<float>(v)));
      }
      halo[cc * DHP + hp] = v;
    }
    __syncthreads();
    for (int cc = 0; cc < nci; ++cc) {
      const TM* hc = halo + cc * DHP + ly * DH + lx;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const TM v = hc[(t / 3) * DH + t % 3];
#pragma unroll
        for (int j = 0; j < DCO; ++j)
          if (j < nco) acc[j] += wl[(static_cast<size_t>(j) * a.CI + c0 + cc) * 9 + t] * v;
      }
    }
  }
  if (!inside) return;
  const TM* bias = static_cast<const TM*>(a.bias);
  const bool sp = a.act == IDQ_ACT_SOFTPLUS;
  for (int j = 0; j < DCO; ++j) {
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
  const int ntx = (a.W + DT - 1) / DT, nty = (a.H + DT - 1) / DT;
  dim3 grid(ntx * nty, a.NI, (a.CO + DCO - 1) / DCO);
  if (grid.y > 65535 || grid.z > 65535) return fail(IDQ_E_INVAL, "too many images in one conv pass");
  const size_t es = prec == PREC_F64 ? 8 : 4;
  const size_t lds = es * (static_cast<size_t>(DCI) * DHP + static_cast<size_t>(DCO) * a.CI * 9);
  if (lds > 64 * 1024) return fail(IDQ_E_UNSUPPORTED, "direct conv: too many input channels");
  if (a.ev0) IDQ_HIP(hipEventRecord(a.ev0, s));
  switch (prec) {
    case PREC_F64:
      conv_direct_kernel<double, double, double, false><<<grid, 256, lds, s>>>(a, ntx);
      break;
    case PREC_F32:
      conv_direct_kernel<float, float, float, false><<<grid, 256, lds, s>>>(a, ntx);
      break;
    case PREC_BF16:
      conv_direct_kernel<float, float, bf16, true><<<grid, 256, lds, s>>>(a, ntx);
      break;
    default:
      return fail(IDQ_E_INVAL, "bad conv precision");
  }
  IDQ_HIP(hipGetLastError());
  if (a.ev1) IDQ_HIP(hipEventRecord(a.ev1, s));
  return IDQ_OK;
}

}  // namespace idq
