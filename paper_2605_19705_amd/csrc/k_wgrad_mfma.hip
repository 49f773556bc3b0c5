// Weight gradient of a 3x3 conv layer on the float32 matrix cores:
//     dW[co][ci][tap] = sum_p G[p][co] * A[p + off(tap)][ci],   db[co] = sum_p G[p][co]
// (the correlations of the parameter gradients of eq. GS's network, App. D.1),
// as a GEMM with M = co, N = (tap, ci) and K = pixels, split over pixel chunks.
//
// A workgroup (4 waves) walks 8 x 16-pixel tiles of the images, one chunk of
// tiles per workgroup.  Per tile it stages G (NHWC, 128 pixels x CO) and the
// (10 x 18)-pixel halo of A (NHWC, CI channels; with the P_JVP prologue the
// operand sigma'(h) * a', sigma' recovered from the stored activation) in LDS,
// zero outside the image, with a 16-byte pad per pixel so the fragment reads
// of the four lane rows fall in different banks.  Wave w owns output-channel
// block w % (CO/16) and a share of the 9 * CI/16 (tap, ci-block) pairs; per
// 4-pixel k step it reads one A fragment (16 co x 4 px of G) and one B
// fragment per pair (4 px x 16 ci of the shifted A), one v_mfma_f32_16x16x4f32
// each, accumulating the whole chunk in registers.  The chunk's sums go to
// float64 partials [chunk][slot] that a fixed-order reduction adds up, so the
// result does not depend on scheduling.  Used for float32 and bf16 passes over
// NHWC activations with CI and CO multiples of 16 (the hidden layers; bf16
// values convert exactly to float32 in LDS, so the products are those of the
// float32 path) and for the image-facing layers of the 32- and 64-channel
// nets, whose 1..16-channel NCHW operand is zero-padded to 16 channels in LDS.
#include "kernels.h"

namespace idq {

namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

constexpr int kWT = 256;             // threads
constexpr int TH = 8, TW = 16;       // output tile
constexpr int HH = TH + 2, HWD = TW + 2, HPIX = HH * HWD, TPIX = TH * TW;

template <int CI, int CO>
struct WCfg {
  static constexpr int NCI = CI / 16, NCO = CO / 16;
  static constexpr int PAIRS = 9 * NCI;              // (tap, ci-block) pairs
  static constexpr int SHARE = 4 / NCO;              // waves per co-block
  static constexpr int MAXP = (PAIRS + SHARE - 1) / SHARE;
  static constexpr int CIP = CI + 4, COP = CO + 4;   // padded pixel strides (floats)
  static constexpr int LDS = (HPIX * CIP + TPIX * COP) * 4;
  static_assert(NCO == 1 || NCO == 2 || NCO == 4, "CO must be 16, 32 or 64");
};

// 4 consecutive NHWC channels as floats: float32 or bfloat16 storage
template <bool BF>
__device__ inline f32x4_t load4(const void* base, size_t e) {
  if (BF) {
    const uint2 u = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(base) + e);
    return f32x4_t{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                   __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u)};
  }
  return *reinterpret_cast<const f32x4_t*>(static_cast<const float*>(base) + e);
}

// CI, CO: the GEMM's (padded) channel counts, multiples of 16.  A_NCHW / G_NCHW:
// the operand is a 1..16-channel NCHW state tensor (an image-facing layer: its
// a.CI / a.CO real channels, zero-padded to 16 in LDS).  BF: the NHWC
// activations are bfloat16 (the warm start's bf16 training), converted exactly
// to float32 in LDS; NCHW state tensors are float32.
template <int CI, int CO, bool A_NCHW, bool G_NCHW, bool BF>
__global__ __launch_bounds__(kWT, 1) void wgrad_mfma_kernel(WgradArgs a, int ntx, int nty,
                                                           int ntiles) {
  using C = WCfg<CI, CO>;
  const int cir = A_NCHW ? a.CI : CI, cor = G_NCHW ? a.CO : CO;
  extern __shared__ __attribute__((aligned(16))) float wsm[];
  float* la = wsm;                    // [HPIX][CIP]
  float* lg = wsm + HPIX * C::CIP;    // [TPIX][COP]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int cbo = wv % C::NCO;        // this wave's output-channel block
  const int p0 = wv / C::NCO;         // its first (tap, ci-block) pair
  const bool sp = a.act == IDQ_ACT_SOFTPLUS;
  const float* G = static_cast<const float*>(a.g);
  const float* A0 = static_cast<const float*>(a.a0);
  const float* A1 = static_cast<const float*>(a.a1);   // NCHW operands only
  f32x4_t acc[C::MAXP];
#pragma unroll
  for (int j = 0; j < C::MAXP; ++j) acc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;                   // bias: thread tid < CO sums channel tid
  const int tiles_per_img = ntx * nty;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int ni = t / tiles_per_img, rem = t - ni * tiles_per_img;
    const int ty0 = (rem / ntx) * TH, tx0 = (rem % ntx) * TW;
    __syncthreads();  // the previous tile's fragments have been read
    if constexpr (A_NCHW) {
      // one value per item; channels past the real ones stay zero
      for (int it = tid; it < HPIX * CI; it += kWT) {
        const int c = it / HPIX, p = it - c * HPIX;
        const int gy = ty0 - 1 + p / HWD, gx = tx0 - 1 + p % HWD;
        float v = 0.f;
        if (c < cir && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
          const size_t e = ((static_cast<size_t>(ni) * cir + c) * a.H + gy) * a.W + gx;
          v = A0[e];
          if (a.a_pro == P_JVP) v = (sp ? dsp_from_a(v) : 1.f) * A1[e];
        }
        la[p * C::CIP + c] = v;
      }
    } else
    // A halo: 4 channels per item
    for (int it = tid; it < HPIX * (CI / 4); it += kWT) {
      const int p = it / (CI / 4), c4 = (it - p * (CI / 4)) * 4;
      const int gy = ty0 - 1 + p / HWD, gx = tx0 - 1 + p % HWD;
      f32x4_t v = {0.f, 0.f, 0.f, 0.f};
      if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
        const size_t e = ((static_cast<size_t>(ni) * a.H + gy) * a.W + gx) * CI + c4;
        v = load4<BF>(a.a0, e);
        if (a.a_pro == P_JVP) {
          const f32x4_t d = load4<BF>(a.a1, e);
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = (sp ? dsp_from_a(v[q]) : 1.f) * d[q];
        }
      }
      *reinterpret_cast<f32x4_t*>(la + p * C::CIP + c4) = v;
    }
    if constexpr (G_NCHW) {
      for (int it = tid; it < TPIX * CO; it += kWT) {
        const int c = it / TPIX, p = it - c * TPIX;
        const int gy = ty0 + p / TW, gx = tx0 + p % TW;
        float v = 0.f;
        if (c < cor && gy < a.H && gx < a.W)
          v = G[((static_cast<size_t>(ni) * cor + c) * a.H + gy) * a.W + gx];
        lg[p * C::COP + c] = v;
      }
    } else
    // G tile
    for (int it = tid; it < TPIX * (CO / 4); it += kWT) {
      const int p = it / (CO / 4), c4 = (it - p * (CO / 4)) * 4;
      const int gy = ty0 + p / TW, gx = tx0 + p % TW;
      f32x4_t v = {0.f, 0.f, 0.f, 0.f};
      if (gy < a.H && gx < a.W)
        v = load4<BF>(a.g, ((static_cast<size_t>(ni) * a.H + gy) * a.W + gx) * CO + c4);
      *reinterpret_cast<f32x4_t*>(lg + p * C::COP + c4) = v;
    }
    __syncthreads();
    if (a.with_bias && tid < cor) {
      for (int p = 0; p < TPIX; ++p) bsum += lg[p * C::COP + tid];
    }
    // K loop: 4 tile pixels per step; lane row kq takes pixel 4s + kq
    for (int s = 0; s < TPIX / 4; ++s) {
      const int px = 4 * s + kq;
      const float af = lg[px * C::COP + cbo * 16 + l16];
      const int py = px / TW, pxx = px - (px / TW) * TW;
#pragma unroll
      for (int j = 0; j < C::MAXP; ++j) {
        const int pr = p0 + j * C::SHARE;
        if (pr < C::PAIRS) {
          const int tap = pr / C::NCI, cb = pr - (pr / C::NCI) * C::NCI;
          const int hp = (py + tap / 3) * HWD + pxx + tap % 3;
          const float bfv = la[hp * C::CIP + cb * 16 + l16];
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bfv, acc[j], 0, 0, 0);
        }
      }
    }
  }
  // partials of this chunk: lane holds D rows (co) 4 kq + i, column (ci) l16
  const int nw = cor * cir * 9;
  const int nslots = nw + (a.with_bias ? cor : 0);
  double* out = a.partials + static_cast<size_t>(blockIdx.x) * nslots;
#pragma unroll
  for (int j = 0; j < C::MAXP; ++j) {
    const int pr = p0 + j * C::SHARE;
    if (pr < C::PAIRS) {
      const int tap = pr / C::NCI, cb = pr - (pr / C::NCI) * C::NCI;
      const int ci = cb * 16 + l16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = cbo * 16 + 4 * kq + i;
        if (ci < cir && co < cor)
          out[(static_cast<size_t>(co) * cir + ci) * 9 + tap] = static_cast<double>(acc[j][i]);
      }
    }
  }
  if (a.with_bias && tid < cor) out[nw + tid] = static_cast<double>(bsum);
}

template <int CI, int CO, bool A_NCHW = false, bool G_NCHW = false, bool BF = false>
int launch_shape(const WgradArgs& a, hipStream_t s) {
  using C = WCfg<CI, CO>;
  static bool attr = false;
  auto kern = wgrad_mfma_kernel<CI, CO, A_NCHW, G_NCHW, BF>;
  if (!attr) {
    IDQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS));
    attr = true;
  }
  const int ntx = (a.W + TW - 1) / TW, nty = (a.H + TH - 1) / TH;
  const long long nt = static_cast<long long>(a.NI) * ntx * nty;
  if (nt > 0x7fffffff) return fail(IDQ_E_INVAL, "too many tiles");
  kern<<<a.nchunk, kWT, C::LDS, s>>>(a, ntx, nty, static_cast<int>(nt));
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

}  // namespace

bool wgrad_mfma_supported(const WgradArgs& a, int prec) {
  if (prec != PREC_F32 && prec != PREC_BF16) return false;
  const int ci = a.CI, co = a.CO;
  // image-facing layers: A an NCHW state tensor (3 -> 32 / 64), or G one (32 / 64 -> 3)
  if (a.a_fmt == F_NCHW && a.g_fmt == F_NHWC) return ci <= 16 && (co == 32 || co == 64);
  if (a.a_fmt == F_NHWC && a.g_fmt == F_NCHW) return (ci == 32 || ci == 64) && co <= 16;
  if (a.g_fmt != F_NHWC || a.a_fmt != F_NHWC) return false;
  return (ci == 16 && co == 16 && prec == PREC_F32) || (ci == 32 && co == 32) ||
         (ci == 64 && co == 64) || (ci == 32 && co == 64) || (ci == 64 && co == 32) ||
         (ci == 96 && co == 32);
}

namespace {
template <bool BF>
int dispatch(const WgradArgs& a, hipStream_t s) {
  if (a.a_fmt == F_NCHW)
    return a.CO == 64 ? launch_shape<16, 64, true, false, BF>(a, s)
                      : launch_shape<16, 32, true, false, BF>(a, s);
  if (a.g_fmt == F_NCHW)
    return a.CI == 64 ? launch_shape<64, 16, false, true, BF>(a, s)
                      : launch_shape<32, 16, false, true, BF>(a, s);
  switch (a.CI * 1000 + a.CO) {
    case 16016: return launch_shape<16, 16, false, false, BF>(a, s);
    case 32032: return launch_shape<32, 32, false, false, BF>(a, s);
    case 64064: return launch_shape<64, 64, false, false, BF>(a, s);
    case 32064: return launch_shape<32, 64, false, false, BF>(a, s);
    case 64032: return launch_shape<64, 32, false, false, BF>(a, s);
    case 96032: return launch_shape<96, 32, false, false, BF>(a, s);
    default: return fail(IDQ_E_UNSUPPORTED, "wgrad: no matrix-core shape");
  }
}
}  // namespace

int launch_wgrad_mfma(const WgradArgs& a, int prec, hipStream_t s) {
  if (a.nchunk <= 0) return fail(IDQ_E_INVAL, "wgrad: no chunks");
  return prec == PREC_BF16 ? dispatch<true>(a, s) : dispatch<false>(a, s);
}

}  // namespace idq
