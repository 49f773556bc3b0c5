// Implicit-GEMM 3x3 convolution on the gfx950 matrix cores.
//
// One pass computes, for every output pixel p and output channel co,
//     acc[co](p) = sum_k Wm[co][k] * X[k](p),   k = tap * CI + ci,
//     X[tap * CI + ci](p) = a[ci](p + (tap / 3 - 1, tap % 3 - 1))   (zero outside)
// as D = Wm (M = co) x X (N = pixels), K = 9 * CI, on 16x16 MFMA tiles:
//   bf16: v_mfma_f32_16x16x32_bf16  (K chunk 32: lane group g owns k 8g..8g+7)
//   fp32: v_mfma_f32_16x16x4_f32    (K chunk 16: lane group g owns k 4g..4g+3 as
//         a float4 whose component s feeds the s-th of four MFMAs; the same
//         k permutation is applied to the weights, so the sum is unchanged)
// Operand / accumulator lane layouts (16x16 tiles): lane l supplies row l%16 of
// A and column l%16 of B for its k slice; it receives D rows 4*(l/16)+i,
// column l%16, i = 0..3.
//
// Work decomposition: a persistent grid of 256-thread workgroups loops over
// 16x16-pixel output tiles (of all net images).  Each tile's (18 x 18)-pixel
// halo tile is staged in LDS (pixel-major, channels contiguous, a 16-byte pad
// per pixel keeps the B-fragment reads conflict-free); wave w computes output
// rows 4w..4w+3 for every output channel.  BF16 weights live in LDS for the
// whole kernel (staged once per workgroup, already in fragment order); FP32
// weights are read in fragment order straight from global memory (their
// matrix-core rate is 1/16 of bf16, so the L2 traffic is small).
// Thin layers (CI <= 4, the image-facing convs) gather their operand from a
// per-pixel 4-channel LDS tile.
#include "kernels.h"

namespace idq {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4_t;

constexpr int kThreads = 256;
constexpr int TH = 16, TW = 16;
constexpr int HW_ = TW + 2, HH_ = TH + 2, NPIX = HW_ * HH_;
constexpr int RW = 4;  // output rows per wave

template <int PREC, int CI, int CO>
struct Cfg {
  static constexpr bool BF = PREC == PREC_BF16;
  static constexpr int ES = BF ? 2 : 4;        // LDS element bytes
  static constexpr int V = BF ? 8 : 4;         // k elements per lane per chunk (16 bytes)
  static constexpr int KC = 4 * V;             // k per chunk
  static constexpr int K = 9 * CI;
  static constexpr int NCH = (K + KC - 1) / KC;
  static constexpr int NJ = (CO + 15) / 16;
  static constexpr bool VEC = (CI % V) == 0;
  static constexpr int CIP = VEC ? CI : 4;
  static constexpr int PIXB = CIP * ES + (VEC ? 16 : 0);
  static constexpr int LDS_IN = (NPIX * PIXB + 15) / 16 * 16;
  static constexpr bool WLDS = BF;
  static constexpr int WBYTES = NCH * NJ * 64 * 16;
  static constexpr int LDS = LDS_IN + (WLDS ? WBYTES : 0);
  // fp32 reads its weights from global memory: a short unroll keeps the
  // hoisted loads within the register file
  static constexpr int UNROLL = BF ? NCH : 2;
};

__device__ inline unsigned pack2(bf16 lo, bf16 hi) {
  return static_cast<unsigned>(lo.u) | (static_cast<unsigned>(hi.u) << 16);
}
__device__ inline float u2f(unsigned u) { return __builtin_bit_cast(float, u); }
__device__ inline unsigned f2u(float f) { return __builtin_bit_cast(unsigned, f); }

template <bool BF>
__device__ inline float lds_scalar(const char* p) {
  if (BF) {
    bf16 v;
    v.u = *reinterpret_cast<const uint16_t*>(p);
    return bf2f(v);
  }
  return *reinterpret_cast<const float*>(p);
}

template <int PREC, int CI, int CO>
__global__ __launch_bounds__(kThreads, 1) void conv_mfma_kernel(ConvArgs a, int ntx, int nty,
                                                               int ntiles) {
  using C = Cfg<PREC, CI, CO>;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  char* lin = smem;
  const u32x4_t* lw = reinterpret_cast<const u32x4_t*>(smem + C::LDS_IN);
  const u32x4_t* gw = static_cast<const u32x4_t*>(a.wmfma);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, c16 = lane & 15;
  const bool sp = a.act == IDQ_ACT_SOFTPLUS;

  if (C::WLDS) {
    u32x4_t* dst = reinterpret_cast<u32x4_t*>(smem + C::LDS_IN);
    for (int i = tid; i < C::NCH * C::NJ * 64; i += kThreads) dst[i] = gw[i];
  }

  const int tiles_per_img = ntx * nty;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int ni = t / tiles_per_img;
    const int rem = t - ni * tiles_per_img;
    const int ty0 = (rem / ntx) * TH, tx0 = (rem % ntx) * TW;
    if (!gate_open(a.gate, a.gate_mask, ni / a.img_div)) continue;
    __syncthreads();
    // ---- stage the (TH+2) x (TW+2) halo tile --------------------------------
    if (C::VEC) {
      constexpr int VPP = CI / C::V;  // 16-byte vectors per pixel
      for (int it = tid; it < NPIX * VPP; it += kThreads) {
        const int p = it / VPP, v = it - (it / VPP) * VPP;
        const int ly = p / HW_, lx = p - (p / HW_) * HW_;
        const int gy = ty0 - 1 + ly, gx = tx0 - 1 + lx;
        u32x4_t val = {0u, 0u, 0u, 0u};
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
          const size_t e = ((static_cast<size_t>(ni) * a.H + gy) * a.W + gx) * CI + v * C::V;
          if (C::BF) {
            const u32x4_t* src = reinterpret_cast<const u32x4_t*>(static_cast<const bf16*>(a.in0) + e);
            val = *src;
            if (a.pro == P_JVP) {
              const u32x4_t hd = *reinterpret_cast<const u32x4_t*>(static_cast<const bf16*>(a.in1) + e);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                bf16 lo, hi, dlo, dhi;
                lo.u = val[q] & 0xffffu;
                hi.u = val[q] >> 16;
                dlo.u = hd[q] & 0xffffu;
                dhi.u = hd[q] >> 16;
                const float s0 = sp ? dsp_from_a_fast(bf2f(lo)) : 1.f;
                const float s1 = sp ? dsp_from_a_fast(bf2f(hi)) : 1.f;
                val[q] = pack2(f2bf(s0 * bf2f(dlo)), f2bf(s1 * bf2f(dhi)));
              }
            }
          } else {
            const f32x4_t* src = reinterpret_cast<const f32x4_t*>(static_cast<const float*>(a.in0) + e);
            f32x4_t fv = *src;
            if (a.pro == P_JVP) {
              const f32x4_t hd = *reinterpret_cast<const f32x4_t*>(static_cast<const float*>(a.in1) + e);
#pragma unroll
              for (int q = 0; q < 4; ++q) fv[q] = (sp ? dsp_from_a(fv[q]) : 1.f) * hd[q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) val[q] = f2u(fv[q]);
          }
        }
        *reinterpret_cast<u32x4_t*>(lin + p * C::PIXB + v * 16) = val;
      }
    } else {
      // image-facing input: float state tensor in NCHW with CI <= 4 planes
      const float* src = static_cast<const float*>(a.in0);
      for (int it = tid; it < NPIX * CI; it += kThreads) {
        const int p = it / CI, ci = it - (it / CI) * CI;
        const int ly = p / HW_, lx = p - (p / HW_) * HW_;
        const int gy = ty0 - 1 + ly, gx = tx0 - 1 + lx;
        float v = 0.f;
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
          v = src[((static_cast<size_t>(ni) * CI + ci) * a.H + gy) * a.W + gx];
        char* d = lin + p * C::PIXB + ci * C::ES;
        if (C::BF)
          *reinterpret_cast<uint16_t*>(d) = f2bf(v).u;
        else
          *reinterpret_cast<float*>(d) = v;
      }
    }
    __syncthreads();
    if (a.work_px && tid == 0) {
      const int vh = a.H - ty0 < TH ? a.H - ty0 : TH, vw = a.W - tx0 < TW ? a.W - tx0 : TW;
      atomicAdd(a.work_px, static_cast<unsigned long long>(vh * vw));
    }
    // ---- K loop on the matrix cores ------------------------------------------
    f32x4_t acc[RW][C::NJ];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int j = 0; j < C::NJ; ++j) acc[r][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll C::UNROLL
    for (int ch = 0; ch < C::NCH; ++ch) {
      const int kb = ch * C::KC + g * C::V;
      u32x4_t af[C::NJ];
#pragma unroll
      for (int j = 0; j < C::NJ; ++j) af[j] = C::WLDS ? lw[(ch * C::NJ + j) * 64 + lane]
                                                   : gw[(ch * C::NJ + j) * 64 + lane];
      u32x4_t bfr[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int row = wv * RW + r;
        if (C::VEC) {
          if (kb < C::K) {
            const int tap = kb / CI, ci0 = kb - (kb / CI) * CI;
            const int pix = (row + tap / 3) * HW_ + c16 + tap % 3;
            bfr[r] = *reinterpret_cast<const u32x4_t*>(lin + pix * C::PIXB + ci0 * C::ES);
          } else {
            bfr[r] = u32x4_t{0u, 0u, 0u, 0u};
          }
        } else {
          float vals[C::V];
#pragma unroll
          for (int e = 0; e < C::V; ++e) {
            const int k = kb + e;
            float v = 0.f;
            if (k < C::K) {
              const int tap = k / CI, ci = k - (k / CI) * CI;
              const int pix = (row + tap / 3) * HW_ + c16 + tap % 3;
              v = lds_scalar<C::BF>(lin + pix * C::PIXB + ci * C::ES);
            }
            vals[e] = v;
          }
          if (C::BF) {
#pragma unroll
            for (int q = 0; q < 4; ++q) bfr[r][q] = pack2(f2bf(vals[2 * q]), f2bf(vals[2 * q + 1]));
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) bfr[r][q] = f2u(vals[q]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < C::NJ; ++j) {
          if (C::BF) {
            acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8_t, af[j]), __builtin_bit_cast(bf16x8_t, bfr[r]), acc[r][j],
                0, 0, 0);
          } else {
#pragma unroll
            for (int s = 0; s < 4; ++s)
              acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(u2f(af[j][s]), u2f(bfr[r][s]),
                                                               acc[r][j], 0, 0, 0);
          }
        }
    }
    // ---- epilogue ----------------------------------------------------------------
    const float* bias = static_cast<const float*>(a.bias);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int oy = ty0 + wv * RW + r, ox = tx0 + c16;
      if (oy >= a.H || ox >= a.W) continue;
#pragma unroll
      for (int j = 0; j < C::NJ; ++j) {
        const int co0 = 16 * j + 4 * g;
        if (co0 >= CO) continue;
        if (a.out_fmt == F_NHWC) {
          const size_t o = ((static_cast<size_t>(ni) * a.H + oy) * a.W + ox) * CO + co0;
          float v[4], w1[4];
          bool two = false;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int co = co0 + i;
            const float x = acc[r][j][i];
            float res = x;
            if (co < CO) {
              switch (a.epi) {
                case E_ACT: {
                  const float hv = x + (bias ? bias[co] : 0.f);
                  res = sp ? (C::BF ? softplus_fast(hv) : softplus_f(hv)) : hv;
                  break;
                }
                case E_DELTA: {
                  const float av = C::BF ? bf2f(static_cast<const bf16*>(a.e0)[o + i])
                                         : static_cast<const float*>(a.e0)[o + i];
                  res = (sp ? (C::BF ? dsp_from_a_fast(av) : dsp_from_a(av)) : 1.f) * x;
                  break;
                }
                case E_DDOT: {
                  // float32 passes only (the HVP is not run in bf16)
                  const float av = static_cast<const float*>(a.e0)[o + i];
                  const float hd = static_cast<const float*>(a.e1)[o + i];
                  const float tv = static_cast<const float*>(a.e2)[o + i];
                  const float s1 = sp ? dsp_from_a(av) : 1.f;
                  const float s2 = sp ? s1 * (1.f - s1) : 0.f;
                  res = s2 * hd * tv + s1 * x;
                  w1[i] = s1 * tv;
                  two = true;
                  break;
                }
                default: break;  // E_RAW
              }
            }
            v[i] = res;
          }
          if (C::BF) {
            bf16* out = static_cast<bf16*>(a.out0) + o;
            if (CO % 4 == 0) {
              uint2 pk;
              pk.x = pack2(f2bf(v[0]), f2bf(v[1]));
              pk.y = pack2(f2bf(v[2]), f2bf(v[3]));
              *reinterpret_cast<uint2*>(out) = pk;
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (co0 + i < CO) out[i] = f2bf(v[i]);
            }
          } else {
            float* out = static_cast<float*>(a.out0) + o;
            if (CO % 4 == 0) {
              *reinterpret_cast<f32x4_t*>(out) = f32x4_t{v[0], v[1], v[2], v[3]};
              if (two)
                *reinterpret_cast<f32x4_t*>(static_cast<float*>(a.out1) + o) =
                    f32x4_t{w1[0], w1[1], w1[2], w1[3]};
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (co0 + i < CO) {
                  out[i] = v[i];
                  if (two) static_cast<float*>(a.out1)[o + i] = w1[i];
                }
            }
          }
        } else {
          // state tensor output in NCHW (float)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int co = co0 + i;
            if (co >= CO) break;
            const size_t o = ((static_cast<size_t>(ni) * CO + co) * a.H + oy) * a.W + ox;
            const float x = acc[r][j][i];
            const float* e0 = static_cast<const float*>(a.e0);
            float res;
            switch (a.epi) {
              case E_RES: res = e0[o] - (x + (bias ? bias[co] : 0.f)); break;
              case E_SUB: res = e0[o] - x; break;
              case E_ACT: {
                const float hv = x + (bias ? bias[co] : 0.f);
                res = sp ? softplus_f(hv) : hv;
                break;
              }
              default: res = x; break;
            }
            static_cast<float*>(a.out0)[o] = res;
          }
        }
      }
    }
  }
}

template <int PREC, int CI, int CO>
int launch_shape(const ConvArgs& a, hipStream_t s) {
  using C = Cfg<PREC, CI, CO>;
  static_assert(C::LDS <= 160 * 1024, "LDS budget");
  static bool attr_set = false;
  static int max_blocks = 0;
  auto kern = conv_mfma_kernel<PREC, CI, CO>;
  if (!attr_set) {
    IDQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS));
    int dev = 0, ncu = 0, occ = 0;
    IDQ_HIP(hipGetDevice(&dev));
    IDQ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    IDQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kThreads, C::LDS));
    if (occ < 1) return fail(IDQ_E_UNSUPPORTED, "MFMA conv does not fit on a compute unit");
    max_blocks = ncu * occ;
    attr_set = true;
  }
  const int ntx = (a.W + TW - 1) / TW, nty = (a.H + TH - 1) / TH;
  const long long nt = static_cast<long long>(a.NI) * ntx * nty;
  if (nt > 0x7fffffff) return fail(IDQ_E_INVAL, "too many tiles");
  const int ntiles = static_cast<int>(nt);
  const int grid = ntiles < max_blocks ? ntiles : max_blocks;
  kern<<<grid, kThreads, C::LDS, s>>>(a, ntx, nty, ntiles);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

// (CI, CO) pairs with an MFMA instantiation: the 3->64->...->64->3 and
// 1->16->16->1 regularizers, the warm-start encoder-decoder, and their
// transposes.
#define IDQ_MFMA_SHAPES(X)                                                                    \
  X(1, 16) X(16, 16) X(16, 1) X(3, 64) X(64, 64) X(64, 3) X(3, 32) X(32, 32) X(32, 64)        \
  X(64, 32) X(96, 32) X(32, 96) X(32, 3)

}  // namespace

bool mfma_supported(int prec, int ci, int co) {
  if (prec != PREC_BF16 && prec != PREC_F32) return false;
#define X(A, B) if (ci == A && co == B) return true;
  IDQ_MFMA_SHAPES(X)
#undef X
  return false;
}

// Weights in fragment order: [chunk][co block j][lane][16 bytes], the lane's
// slice being co = 16 j + lane % 16 and k = chunk * KC + (lane / 16) * V + e.
size_t pack_mfma_weights(int prec, int ci, int co, const double* w, void* dst) {
  const bool bf = prec == PREC_BF16;
  const int V = bf ? 8 : 4, KC = 4 * V, K = 9 * ci;
  const int nch = (K + KC - 1) / KC, nj = (co + 15) / 16;
  const size_t bytes = static_cast<size_t>(nch) * nj * 64 * 16;
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
          if (bf)
            static_cast<bf16*>(dst)[idx] = f2bf(static_cast<float>(v));
          else
            static_cast<float*>(dst)[idx] = static_cast<float>(v);
        }
  return bytes;
}

int launch_conv_mfma(const ConvArgs& a, int prec, hipStream_t s) {
#define X(A, B)                                                                   \
  if (a.CI == A && a.CO == B)                                                     \
    return prec == PREC_BF16 ? launch_shape<PREC_BF16, A, B>(a, s) : launch_shape<PREC_F32, A, B>(a, s);
  IDQ_MFMA_SHAPES(X)
#undef X
  return fail(IDQ_E_UNSUPPORTED, "no MFMA instantiation for this shape");
}

}  // namespace idq
