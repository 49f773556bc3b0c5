// Implicit-GEMM 3x3 convolution on the gfx950 matrix cores (kernel template;
// instantiated per arithmetic in k_conv_mfma_bf16.hip / k_conv_mfma_f32.hip).
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
// Work decomposition: a persistent grid of 256-thread workgroups walks the
// 16x16-pixel output tiles of all images.  Each tile's (18 x 18)-pixel halo
// tile sits in LDS (pixel-major, channels contiguous, a 16-byte pad per pixel
// keeps the B-fragment reads conflict-free); wave w computes output rows
// 4w..4w+3 for every output channel.  While a tile is computed, the next
// tile's halo is already being fetched from HBM into registers, so global
// latency overlaps the matrix-core work.  When a K chunk never straddles two
// taps (CI a multiple of the chunk), the B fragments of one input row are
// loaded once and reused by the three kernel rows (dy) that read it.
// BF16 weights live in LDS for the whole kernel (staged once per workgroup,
// already in fragment order); FP32 weights are read in fragment order from
// global memory (their matrix-core rate is 1/16 of bf16, so L2 traffic is
// small).  Thin layers (CI <= 4, the image-facing convs) gather their operand
// from a per-pixel 4-channel LDS tile.
#pragma once

#include <hip/hip_ext.h>

#include <type_traits>

#include "kernels.h"

namespace idq {
namespace mfma {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4_t;

constexpr int TH = 16, TW = 16;
constexpr int HW_ = TW + 2, HH_ = TH + 2, NPIX = HW_ * HH_;

template <int PREC, int CI, int CO, int PRO = P_NONE>
struct Cfg {
  static constexpr bool BF = PREC == PREC_BF16;      // bf16 activations in HBM
  static constexpr bool SPLIT = PREC == PREC_SPLIT;  // float activations, hi/lo bf16 operands
  static constexpr bool MBF = BF || SPLIT;           // bf16 matrix-core operands
  static constexpr int GES = BF ? 2 : 4;       // HBM activation element bytes
  static constexpr int GV = 16 / GES;          // HBM elements per 16-byte load
  static constexpr int ES = MBF ? 2 : 4;       // LDS element bytes
  static constexpr int V = MBF ? 8 : 4;        // k elements per lane per chunk (16 bytes)
  static constexpr int KC = 4 * V;             // k per chunk
  static constexpr int K = 9 * CI;
  static constexpr int NCH = (K + KC - 1) / KC;
  static constexpr int NJ = (CO + 15) / 16;
  static constexpr bool VEC = (CI % V) == 0;
  static constexpr bool ROWS = (CI % KC) == 0;  // chunks align with taps: reuse rows
  static constexpr int CPT = ROWS ? CI / KC : 0;  // chunks per tap
  static constexpr int CIP = VEC ? CI : 4;
  // split: a pixel holds the hi parts of its channels, then the lo parts
  static constexpr int LO_OFF = CIP * ES;
  static constexpr int PIXB = (SPLIT ? 2 : 1) * CIP * ES + (VEC ? 16 : 0);
  static constexpr int LDS_IN = (NPIX * PIXB + 15) / 16 * 16;
  // launch shape: 4 waves of 4 output rows, one workgroup per tile.  Split
  // passes over 64 input channels, and float32 passes from 3 or 64 channels to
  // 64, run 8 waves of 2 rows instead (two waves per SIMD, so one wave's
  // matrix-core work overlaps the other's staging and epilogue).  For 64 -> 64
  // two workgroups per tile each take half of the output channels, so that the
  // weight fragments of that half (hi and lo for split) fit in LDS beside the
  // tile.  The float32 64-channel tangent pass keeps the 4-wave form: its
  // doubled staging registers would spill at two waves per SIMD.
  static constexpr bool F32W = PREC == PREC_F32 && CO == 64 &&
                               (CI <= 4 || (CI == 64 && PRO == P_NONE));
  static constexpr bool W8 = (SPLIT && CI == 64) || F32W;
  static constexpr int WAVES = W8 ? 8 : 4;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int RWV = TH / WAVES;         // output rows per wave
  static constexpr int CSPLIT = (W8 && CI == 64 && CO == 64) ? 2 : 1;  // workgroups per tile
  static constexpr int NJW = NJ / CSPLIT;        // 16-channel blocks per workgroup
  static constexpr int WBYTES = NCH * NJW * 64 * 16;
  // weight fragments in LDS: always for bf16 operands (hi parts for split);
  // float32 ones where they fit beside the tile (else they come from L2, where
  // a wait for one also waits for the halo and epilogue loads issued before it)
  static constexpr bool WLDS = MBF || LDS_IN + WBYTES <= 160 * 1024;
  // split lo fragments in LDS too where they fit, else read from L2 (where a
  // wait for one also waits for the next tile's halo loads issued before it)
  static constexpr bool WLO_LDS = SPLIT && LDS_IN + 2 * WBYTES <= 160 * 1024;
  static constexpr int LDS = LDS_IN + (WLDS ? WBYTES * (WLO_LDS ? 2 : 1) : 0);
  // prefetch: 16-byte items (VEC) or floats (gather) per thread for one tile
  static constexpr int VPP = VEC ? CI / GV : 0;
  static constexpr int ITEMS = VEC ? (NPIX * VPP + THREADS - 1) / THREADS
                                   : (NPIX * CI + THREADS - 1) / THREADS;
  // fp32 reads its weights from global memory: a short unroll keeps the
  // hoisted loads within the register file
  static constexpr int UNROLL = MBF ? NCH : 2;
  // (dx, chunk) groups of the row-reuse loop unrolled at once: all of them for
  // bf16; one for split operands, whose doubled fragments would spill otherwise
  static constexpr int RUNROLL = BF ? 3 * CPT : 1;
  static_assert(!SPLIT || (VEC && ROWS), "split operands need whole K chunks per tap");
  static_assert(NJ % CSPLIT == 0 && TH % WAVES == 0, "launch shape");
};

__device__ inline unsigned pack2(bf16 lo, bf16 hi) {
  return static_cast<unsigned>(lo.u) | (static_cast<unsigned>(hi.u) << 16);
}
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;
typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2_t;
// two floats -> packed bf16 pair (round to nearest even, v_cvt_pk_bf16_f32)
__device__ inline unsigned pk_bf16(float lo, float hi) {
  const f32x2_t v = {lo, hi};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
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

// Registers holding one tile's halo between its global load and its LDS store.
template <class C, int PRO>
struct Prefetch {
  u32x4_t v[C::VEC ? C::ITEMS : 1];
  u32x4_t w[(C::VEC && PRO == P_JVP) ? C::ITEMS : 1];
  float s[C::VEC ? 1 : C::ITEMS];
};

// Epilogue operand of one tile (E_DELTA): 4 channels per (row, channel block).
template <class C>
struct EpiPrefetch {
  u32x4_t v[C::RWV][C::NJW];
};

template <class C, int CI, int PRO>
__device__ inline void load_tile(const ConvArgs& a, Prefetch<C, PRO>& pf, int ni, int ty0,
                                 int tx0, int tid) {
#pragma unroll
  for (int k = 0; k < C::ITEMS; ++k) {
    const int it = tid + k * C::THREADS;
    if (C::VEC) {
      u32x4_t val = {0u, 0u, 0u, 0u}, hd = {0u, 0u, 0u, 0u};
      if (it < NPIX * C::VPP) {
        const int p = it / C::VPP, v = it - (it / C::VPP) * C::VPP;
        const int ly = p / HW_, lx = p - (p / HW_) * HW_;
        const int gy = ty0 - 1 + ly, gx = tx0 - 1 + lx;
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
          const size_t e = (((static_cast<size_t>(ni) * a.H + gy) * a.W + gx) * CI + v * C::GV) * C::GES;
          val = *reinterpret_cast<const u32x4_t*>(static_cast<const char*>(a.in0) + e);
          if (PRO == P_JVP) hd = *reinterpret_cast<const u32x4_t*>(static_cast<const char*>(a.in1) + e);
        }
      }
      pf.v[k] = val;
      if (PRO == P_JVP) pf.w[k] = hd;
    } else {
      float val = 0.f;
      if (it < NPIX * CI) {
        const int p = it / CI, ci = it - (it / CI) * CI;
        const int ly = p / HW_, lx = p - (p / HW_) * HW_;
        const int gy = ty0 - 1 + ly, gx = tx0 - 1 + lx;
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
          val = static_cast<const float*>(a.in0)[((static_cast<size_t>(ni) * CI + ci) * a.H + gy) * a.W + gx];
      }
      pf.s[k] = val;
    }
  }
}

template <class C, int CI, int PRO>
__device__ inline void store_tile(const ConvArgs& a, const Prefetch<C, PRO>& pf, char* lin,
                                  int tid) {
  const bool sp = a.act == IDQ_ACT_SOFTPLUS;
#pragma unroll
  for (int k = 0; k < C::ITEMS; ++k) {
    const int it = tid + k * C::THREADS;
    if (C::VEC) {
      if (it < NPIX * C::VPP) {
        const int p = it / C::VPP, v = it - (it / C::VPP) * C::VPP;
        u32x4_t val = pf.v[k];
        if (PRO == P_JVP) {
          const u32x4_t hd = pf.w[k];
          if (C::BF) {
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
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              val[q] = f2u((sp ? dsp_from_a(u2f(val[q])) : 1.f) * u2f(hd[q]));
          }
        }
        if (C::SPLIT) {
          // 4 floats -> bf16 hi parts and the bf16-rounded remainders x - hi
          const unsigned h01 = pk_bf16(u2f(val[0]), u2f(val[1]));
          const unsigned h23 = pk_bf16(u2f(val[2]), u2f(val[3]));
          const unsigned l01 = pk_bf16(u2f(val[0]) - u2f(h01 << 16),
                                       u2f(val[1]) - u2f(h01 & 0xffff0000u));
          const unsigned l23 = pk_bf16(u2f(val[2]) - u2f(h23 << 16),
                                       u2f(val[3]) - u2f(h23 & 0xffff0000u));
          *reinterpret_cast<uint2*>(lin + p * C::PIXB + v * 8) = uint2{h01, h23};
          *reinterpret_cast<uint2*>(lin + p * C::PIXB + C::LO_OFF + v * 8) = uint2{l01, l23};
        } else {
          *reinterpret_cast<u32x4_t*>(lin + p * C::PIXB + v * 16) = val;
        }
      }
    } else {
      if (it < NPIX * CI) {
        const int p = it / CI, ci = it - (it / CI) * CI;
        char* d = lin + p * C::PIXB + ci * C::ES;
        if (C::BF)
          *reinterpret_cast<uint16_t*>(d) = f2bf(pf.s[k]).u;
        else
          *reinterpret_cast<float*>(d) = pf.s[k];
      }
    }
  }
}

template <class C>
__device__ inline void mma(f32x4_t& acc, const u32x4_t& af, const u32x4_t& bf) {
  if (C::MBF) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, af),
                                                  __builtin_bit_cast(bf16x8_t, bf), acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(u2f(af[s]), u2f(bf[s]), acc, 0, 0, 0);
  }
}

// Output of one (row r, channel block j) piece of a tile: the lane's 4 output
// channels 16 j + 4 g .. + 3 at pixel (ty0 + 4 wv + r, tx0 + c16).
template <class C, int CO, int EPI>
__device__ inline void epilogue_piece(const ConvArgs& a, const f32x4_t& accv,
                                      const u32x4_t& e0pre, const float (&bias4)[4], int ni,
                                      int ty0, int tx0, int wv, int r, int j, int g, int c16,
                                      bool sp) {
  const int oy = ty0 + wv * C::RWV + r, ox = tx0 + c16;
  if (oy >= a.H || ox >= a.W) return;
  const int co0 = 16 * j + 4 * g;
  if (co0 >= CO) return;
  constexpr bool pre_e0 = EPI == E_DELTA && CO % 4 == 0;
  if constexpr (EPI != E_RES && EPI != E_SUB && EPI != E_ADD) {
    const size_t o = ((static_cast<size_t>(ni) * a.H + oy) * a.W + ox) * CO + co0;
    float v[4], w1[4];
    f32x4_t dd0 = {0.f, 0.f, 0.f, 0.f}, dd1 = dd0, dd2 = dd0;
    bool two = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = co0 + i;
      const float x = accv[i];
      float res = x;
      w1[i] = 0.f;
      if (co < CO) {
        if constexpr (EPI == E_ACT) {
          const float hv = x + bias4[i];
          res = sp ? (C::BF ? softplus_fast(hv) : softplus_hw(hv)) : hv;
        } else if constexpr (EPI == E_DELTA) {
          float av;
          if (pre_e0) {
            if (C::BF) {
              bf16 hb;
              hb.u = static_cast<uint16_t>(e0pre[i >> 1] >> ((i & 1) * 16));
              av = bf2f(hb);
            } else {
              av = u2f(e0pre[i]);
            }
          } else {
            av = C::BF ? bf2f(static_cast<const bf16*>(a.e0)[o + i])
                       : static_cast<const float*>(a.e0)[o + i];
          }
          res = (sp ? (C::BF ? dsp_from_a_fast(av) : dsp_from_a_hw(av)) : 1.f) * x;
        } else if constexpr (EPI == E_DDOT) {
          // float32 passes only (the HVP is not run in bf16)
          if (CO % 4 == 0 && i == 0) {
            dd0 = *reinterpret_cast<const f32x4_t*>(static_cast<const float*>(a.e0) + o);
            dd1 = *reinterpret_cast<const f32x4_t*>(static_cast<const float*>(a.e1) + o);
            dd2 = *reinterpret_cast<const f32x4_t*>(static_cast<const float*>(a.e2) + o);
          }
          const float av = CO % 4 == 0 ? dd0[i] : static_cast<const float*>(a.e0)[o + i];
          const float hd = CO % 4 == 0 ? dd1[i] : static_cast<const float*>(a.e1)[o + i];
          const float tv = CO % 4 == 0 ? dd2[i] : static_cast<const float*>(a.e2)[o + i];
          const float s1 = sp ? dsp_from_a(av) : 1.f;
          const float s2 = sp ? s1 * (1.f - s1) : 0.f;
          res = s2 * hd * tv + s1 * x;
          w1[i] = s1 * tv;
          two = true;
        }
      }
      v[i] = res;
    }
    if (C::BF) {
      bf16* out = static_cast<bf16*>(a.out0) + o;
      if (CO % 4 == 0) {
        uint2 pk;
        pk.x = pk_bf16(v[0], v[1]);
        pk.y = pk_bf16(v[2], v[3]);
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
      const float x = accv[i];
      const float* e0 = static_cast<const float*>(a.e0);
      float res;
      if constexpr (EPI == E_RES)
        res = e0[o] - (x + bias4[i]);
      else if constexpr (EPI == E_ADD)
        res = e0[o] + (x + bias4[i]);
      else
        res = e0[o] - x;
      static_cast<float*>(a.out0)[o] = res;
    }
  }
}

// Buffer resource over `bytes` bytes at `base` (raw addressing, gfx9 word 3);
// a store whose offset is at or beyond `bytes` is dropped by the hardware.
__device__ inline __amdgpu_buffer_rsrc_t out_rsrc(void* base, unsigned bytes) {
  // the arguments are workgroup-uniform; say so, or the compiler wraps every
  // store in a loop over the distinct resources of the wave
  const uint64_t p = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(p));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(p >> 32));
  const uint32_t n = __builtin_amdgcn_readfirstlane(bytes);
  return __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo), static_cast<short>(0),
      static_cast<int>(n), 0x00020000);
}
constexpr unsigned kDropOffset = 0x80000000u;  // beyond every resource we build

typedef __attribute__((ext_vector_type(2))) unsigned u32x2_v;

// Branch-free output piece of the pipelined bf16 kernels (NHWC bf16 output,
// CO a multiple of 16): lanes outside the image store to kDropOffset, and a
// resource of zero bytes (no previous tile yet) drops every store, so the
// piece is one straight run of VALU work that can sit between the MFMAs.
typedef __attribute__((ext_vector_type(4))) unsigned u32x4_v;

template <class C, int CO, int EPI>
__device__ inline void epilogue_piece_pipe(const ConvArgs& a, __amdgpu_buffer_rsrc_t rs,
                                           const f32x4_t& accv, const u32x4_t& e0pre,
                                           const float (&bias4)[4], int ty0, int tx0, int wv,
                                           int r, int j, int g, int c16, bool sp) {
  static_assert((C::BF || C::SPLIT) && CO % 16 == 0, "pipelined pieces store NHWC rows");
  (void)sp;  // SoftPlus only: passes of other activations take other kernels
  const int ly = wv * C::RWV + r, oy = ty0 + ly, ox = tx0 + c16;
  const int co0 = 16 * j + 4 * g;
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float x = accv[i];
    if constexpr (EPI == E_ACT) {
      const float hv = x + bias4[i];
      v[i] = C::BF ? softplus_fast(hv) : softplus_hw(hv);
    } else if constexpr (EPI == E_DELTA) {
      const float av = C::BF ? u2f((e0pre[i >> 1] << ((i & 1) ? 0 : 16)) & 0xffff0000u)
                             : u2f(e0pre[i]);
      v[i] = (C::BF ? dsp_from_a_fast(av) : dsp_from_a_hw(av)) * x;
    } else {
      v[i] = x;
    }
  }
  const bool ok = oy < a.H && ox < a.W;
  const unsigned eb = C::BF ? 2u : 4u;
  const unsigned off = ok ? (static_cast<unsigned>(ly * a.W + ox) * CO + co0) * eb : kDropOffset;
  if constexpr (C::BF) {
    const u32x2_v pk = {pk_bf16(v[0], v[1]), pk_bf16(v[2], v[3])};
    __builtin_amdgcn_raw_buffer_store_b64(pk, rs, static_cast<int>(off), 0, 0);
  } else {
    const u32x4_v pk = {f2u(v[0]), f2u(v[1]), f2u(v[2]), f2u(v[3])};
    __builtin_amdgcn_raw_buffer_store_b128(pk, rs, static_cast<int>(off), 0, 0);
  }
}

template <int PREC, int CI, int CO, int PRO, int EPI>
__global__ __launch_bounds__((Cfg<PREC, CI, CO, PRO>::THREADS), 1) void conv_mfma_kernel(
    ConvArgs a, int ntx, int nty, int ntiles) {
  using C = Cfg<PREC, CI, CO, PRO>;
  static_assert(!C::SPLIT || PRO == P_NONE, "split passes take plain operands");
  // bf16 row-reuse kernels run software-pipelined: the epilogue of the previous
  // tile is issued in pieces between the matrix-core groups of the current one,
  // so its VALU work (SoftPlus / sigma', packing, stores) executes while the
  // MFMAs are in flight instead of after them
  // (bf16 only: the 8-wave split shape already overlaps one wave's epilogue
  // with the other's matrix-core work, and pieces there measured slower)
  constexpr bool PIPE = C::ROWS && C::BF && CO % 16 == 0 &&
                        (EPI == E_ACT || EPI == E_DELTA || EPI == E_RAW);
  constexpr int RW = C::RWV, NJW = C::NJW;
  constexpr int NPIECE = RW * NJW;
  constexpr bool pre_e0 = EPI == E_DELTA && CO % 4 == 0;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  char* lin = smem;
  const u32x4_t* lw = reinterpret_cast<const u32x4_t*>(smem + C::LDS_IN);
  const u32x4_t* lwl = lw + C::NCH * NJW * 64;     // split lo fragments in LDS (WLO_LDS)
  const u32x4_t* gw = static_cast<const u32x4_t*>(a.wmfma);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, c16 = lane & 15;
  const bool sp = a.act == IDQ_ACT_SOFTPLUS;
  const int tiles_per_img = ntx * nty;
  auto open = [&](int t) {
    return gate_open_uniform(a.gate, a.gate_mask, (t / tiles_per_img) / a.img_div);
  };

  // channel group of this workgroup and its walk over the tiles.  Workgroups
  // go to the 8 XCDs round-robin by index, each XCD with its own L2: the
  // channel groups of one tile are blocks b and b + 8 (same XCD), so the second
  // read of the halo tile can hit that L2 (when the grid is a multiple of 16)
  int jh = 0, walker = static_cast<int>(blockIdx.x);
  if (C::CSPLIT > 1) {
    const int b = static_cast<int>(blockIdx.x);
    if (gridDim.x % (8 * C::CSPLIT) == 0) {
      const int grp = b / 8;
      jh = grp % C::CSPLIT;
      walker = (grp / C::CSPLIT) * 8 + b % 8;
    } else {
      jh = b % C::CSPLIT;
      walker = b / C::CSPLIT;
    }
  }
  const int tstep = static_cast<int>(gridDim.x) / C::CSPLIT;
  // first open tile of this workgroup (uniform across it); a workgroup with
  // none leaves before staging weights, so a pass whose images are all in
  // another precision phase costs little more than its launch
  int t = walker;
  while (t < ntiles && !open(t)) t += tstep;
  if (t >= ntiles) return;

  // the first tile's halo is requested before the weights, and the weight
  // fragments are fetched in batches of WB loads per thread before any is
  // written to LDS, so the L2 round trips of the prologue overlap
  auto next_open = [&](int tt) {
    tt += tstep;
    while (tt < ntiles && !open(tt)) tt += tstep;
    return tt;
  };
  auto issue = [&](Prefetch<C, PRO>& p, int tt) {
    if (tt < ntiles) {
      const int ni = tt / tiles_per_img, rem = tt - ni * tiles_per_img;
      load_tile<C, CI, PRO>(a, p, ni, (rem / ntx) * TH, (rem % ntx) * TW, tid);
    }
  };
  // halos in registers ahead of the LDS stage: one tile, or two for the 8-wave
  // shapes (split, and float32 from 3 or 64 channels), whose matrix-core work
  // per tile is short next to the HBM latency of the next halo and whose
  // second buffer fits the register budget
  constexpr int DEPTH = (C::W8 && !C::SPLIT) ? 2 : 1;
  Prefetch<C, PRO> pf, pf2;
  int t1 = DEPTH > 1 ? next_open(t) : 0;
  issue(pf, t);
  if (DEPTH > 1) issue(pf2, t1);
  if (C::WLDS) {
    // LDS fragment i = (ch * NJW + jj) * 64 + lane of this workgroup's channel
    // blocks; the lo parts (WLO_LDS) follow the hi parts
    constexpr int NW = C::NCH * NJW * 64;            // 16-byte fragments per part
    constexpr int NT = NW * (C::WLO_LDS ? 2 : 1);
    constexpr int PER = (NT + C::THREADS - 1) / C::THREADS;
    constexpr int WB = PER < 24 ? PER : 24;
    u32x4_t* dst = reinterpret_cast<u32x4_t*>(smem + C::LDS_IN);
    auto src = [&](int i) {
      const int part = i >= NW ? 1 : 0, f = i - part * NW;
      const int ln = f % 64, jj = (f / 64) % NJW, ch = f / (64 * NJW);
      return (part * C::NCH * C::NJ + ch * C::NJ + jh * NJW + jj) * 64 + ln;
    };
    for (int b0 = 0; b0 < PER; b0 += WB) {
      u32x4_t wbuf[WB];
#pragma unroll
      for (int q = 0; q < WB; ++q) {
        const int i = tid + (b0 + q) * C::THREADS;
        if (i < NT) wbuf[q] = gw[src(i)];
      }
#pragma unroll
      for (int q = 0; q < WB; ++q) {
        const int i = tid + (b0 + q) * C::THREADS;
        if (i < NT) dst[i] = wbuf[q];
      }
    }
  }

  // bias of the output channels this lane owns in the epilogue
  float bias_r[NJW][4];
  {
    const float* bias = static_cast<const float*>(a.bias);
#pragma unroll
    for (int jj = 0; jj < NJW; ++jj)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = 16 * (jh * NJW + jj) + 4 * g + i;
        bias_r[jj][i] = (bias && co < CO) ? bias[co] : 0.f;
      }
  }

  // the previous tile (PIPE): accumulators, epilogue operand, position and
  // the output resource over its rows (none before the first tile)
  f32x4_t accp[PIPE ? RW : 1][PIPE ? NJW : 1];
  EpiPrefetch<C> epp;
  int pty0 = 0, ptx0 = 0;
  __amdgpu_buffer_rsrc_t prs = out_rsrc(a.out0, 0u);
  auto piece_prev = [&](int k) {
    if constexpr (PIPE) {
      if (k < NPIECE) {
        const int r = k / NJW, jj = k % NJW;
        epilogue_piece_pipe<C, CO, EPI>(a, prs, accp[r][jj], epp.v[r][jj], bias_r[jj], pty0,
                                        ptx0, wv, r, jh * NJW + jj, g, c16, sp);
      }
    }
  };

  // one tile: stage its halo from `pcur` into LDS, refill `pcur` with the halo
  // of tile `tfill` (DEPTH tiles ahead), then the K loop and the epilogue
  auto tile = [&](Prefetch<C, PRO>& pcur, const int t, const int tfill) {
    const int ni = t / tiles_per_img;
    const int rem = t - ni * tiles_per_img;
    const int ty0 = (rem / ntx) * TH, tx0 = (rem % ntx) * TW;
    __syncthreads();  // the previous tile's fragments have been read
    store_tile<C, CI, PRO>(a, pcur, lin, tid);
    __syncthreads();
    issue(pcur, tfill);
    if (a.work_px && tid == 0 && jh == 0) {
      const int vh = a.H - ty0 < TH ? a.H - ty0 : TH, vw = a.W - tx0 < TW ? a.W - tx0 : TW;
      atomicAdd(a.work_px, static_cast<unsigned long long>(vh * vw));
    }
    // the epilogue's sigma(h) operand of this tile, fetched now so that its
    // latency hides behind the matrix-core work
    EpiPrefetch<C> ep;
    if (pre_e0) {
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int oy = ty0 + wv * RW + r, ox = tx0 + c16;
#pragma unroll
        for (int jj = 0; jj < NJW; ++jj) {
          const int co0 = 16 * (jh * NJW + jj) + 4 * g;
          ep.v[r][jj] = u32x4_t{0u, 0u, 0u, 0u};
          if (oy < a.H && ox < a.W && co0 < CO) {
            const size_t o = ((static_cast<size_t>(ni) * a.H + oy) * a.W + ox) * CO + co0;
            if (C::BF) {
              const uint2 u = *reinterpret_cast<const uint2*>(static_cast<const bf16*>(a.e0) + o);
              ep.v[r][jj] = u32x4_t{u.x, u.y, 0u, 0u};
            } else {
              ep.v[r][jj] = *reinterpret_cast<const u32x4_t*>(static_cast<const float*>(a.e0) + o);
            }
          }
        }
      }
    }
    // ---- K loop on the matrix cores ------------------------------------------
    f32x4_t acc[RW][NJW];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int j = 0; j < NJW; ++j) acc[r][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    if constexpr (C::ROWS) {
      // k = (dy*3 + dx) * CI + c*KC + slice: load the RW+2 input rows once per
      // (dx, c) and reuse them for dy = 0, 1, 2.  The weight fragments of the
      // next (dx, c, dy) group are fetched while the current group's MFMAs
      // run (for fp32 they come from L2, whose latency would otherwise stall
      // every group).
      constexpr int NL = C::SPLIT ? NJW : 1;
      const u32x4_t* gwl = gw + C::NCH * C::NJ * 64;  // split: lo fragments in L2
      // fragments of this workgroup's channel blocks: LDS holds only those
      // (index ch * NJW + jj); global memory holds all NJ (CSPLIT is 1 there)
      auto load_af = [&](u32x4_t* dst, u32x4_t* dlo, int dxc, int dy) {
        const int ch = (dy * 3 + dxc / C::CPT) * C::CPT + dxc % C::CPT;
#pragma unroll
        for (int j = 0; j < NJW; ++j) dst[j] = C::WLDS ? lw[(ch * NJW + j) * 64 + lane]
                                                    : gw[(ch * C::NJ + j) * 64 + lane];
        if (C::SPLIT) {
#pragma unroll
          for (int j = 0; j < NJW; ++j) dlo[j] = C::WLO_LDS ? lwl[(ch * NJW + j) * 64 + lane]
                                                         : gwl[(ch * C::NJ + j) * 64 + lane];
        }
      };
      u32x4_t afc[NJW], afn[NJW], alc[NL], aln[NL];
      load_af(afc, alc, 0, 0);
      // one (dx, chunk) step: its RW+2 input rows, then the three dy groups;
      // WITH_PIECES puts a piece of the previous tile's epilogue after each group
      auto dxc_step = [&](int dxc, auto with_pieces) {
        const int dx = dxc / C::CPT, c = dxc % C::CPT;
        u32x4_t brow[RW + 2], browl[C::SPLIT ? RW + 2 : 1];
        const int coff = (c * C::KC + g * C::V) * C::ES;
#pragma unroll
        for (int ir = 0; ir < RW + 2; ++ir) {
          const int pix = (wv * RW + ir) * HW_ + c16 + dx;
          brow[ir] = *reinterpret_cast<const u32x4_t*>(lin + pix * C::PIXB + coff);
          if (C::SPLIT)
            browl[ir] = *reinterpret_cast<const u32x4_t*>(lin + pix * C::PIXB + C::LO_OFF + coff);
        }
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          if (dy < 2)
            load_af(afn, aln, dxc, dy + 1);
          else if (dxc + 1 < 3 * C::CPT)
            load_af(afn, aln, dxc + 1, 0);
          // split: small terms first (lo*hi, hi*lo, then hi*hi), each term over
          // all accumulators before the next, so consecutive MFMAs never wait
          // for one another's result
          if (C::SPLIT) {
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
              for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], afc[j], browl[r + dy]);
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
              for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], alc[j], brow[r + dy]);
          }
#pragma unroll
          for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], afc[j], brow[r + dy]);
          if constexpr (decltype(with_pieces)::value) piece_prev(dxc * 3 + dy);
#pragma unroll
          for (int j = 0; j < NJW; ++j) afc[j] = afn[j];
          if (C::SPLIT) {
#pragma unroll
            for (int j = 0; j < NJW; ++j) alc[j] = aln[j];
          }
        }
      };
      if constexpr (C::SPLIT) {
        // split operands: the input rows (hi and lo parts) of the next (dx, chunk)
        // step are read from LDS before this step's matrix-core groups, so their
        // latency hides behind 36 MFMAs instead of stalling the first group
        constexpr int NR = RW + 2;
        u32x4_t bh[2][NR], bl[2][NR];
        auto load_rows = [&](u32x4_t* h, u32x4_t* l, int dxc) {
          const int dx = dxc / C::CPT, c = dxc % C::CPT;
          const int coff = (c * C::KC + g * C::V) * C::ES;
#pragma unroll
          for (int ir = 0; ir < NR; ++ir) {
            const int pix = (wv * RW + ir) * HW_ + c16 + dx;
            h[ir] = *reinterpret_cast<const u32x4_t*>(lin + pix * C::PIXB + coff);
            l[ir] = *reinterpret_cast<const u32x4_t*>(lin + pix * C::PIXB + C::LO_OFF + coff);
          }
        };
        // one (dx, chunk) step on the rows in (h, l) while (hn, ln) receive the next
        // step's rows; steps run in pairs so that both buffers are fixed registers
        auto split_step = [&](int dxc, const u32x4_t* h, const u32x4_t* l, u32x4_t* hn,
                              u32x4_t* ln) {
          if (dxc + 1 < 3 * C::CPT) load_rows(hn, ln, dxc + 1);
#pragma unroll
          for (int dy = 0; dy < 3; ++dy) {
            if (dy < 2)
              load_af(afn, aln, dxc, dy + 1);
            else if (dxc + 1 < 3 * C::CPT)
              load_af(afn, aln, dxc + 1, 0);
            // the scheduler may not sink these reads into the matrix-core group
            // below: issued here, their latency hides behind its 12 MFMAs
            __builtin_amdgcn_sched_barrier(0);
            // small terms first (lo*hi, hi*lo, then hi*hi), each term over all
            // accumulators before the next
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
              for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], afc[j], l[r + dy]);
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
              for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], alc[j], h[r + dy]);
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
              for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], afc[j], h[r + dy]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < NJW; ++j) {
              afc[j] = afn[j];
              alc[j] = aln[j];
            }
          }
        };
        constexpr int NS = 3 * C::CPT;
        load_rows(bh[0], bl[0], 0);
#pragma unroll 1
        for (int dxc = 0; dxc + 1 < NS; dxc += 2) {
          split_step(dxc, bh[0], bl[0], bh[1], bl[1]);
          split_step(dxc + 1, bh[1], bl[1], bh[0], bl[0]);
        }
        if constexpr (NS % 2 == 1) split_step(NS - 1, bh[0], bl[0], bh[1], bl[1]);
      } else {
      // the first PEEL steps (unrolled: their piece indices are constants) carry
      // the previous tile's epilogue pieces; the rest run as a plain loop
      constexpr int PEEL = PIPE ? ((NPIECE + 2) / 3 < 3 * C::CPT ? (NPIECE + 2) / 3 : 3 * C::CPT) : 0;
#pragma unroll
      for (int dxc = 0; dxc < PEEL; ++dxc) dxc_step(dxc, std::true_type{});
#pragma unroll C::RUNROLL
      for (int dxc = PEEL; dxc < 3 * C::CPT; ++dxc) dxc_step(dxc, std::false_type{});
      }
    } else {
#pragma unroll C::UNROLL
      for (int ch = 0; ch < C::NCH; ++ch) {
        const int kb = ch * C::KC + g * C::V;
        static_assert(C::CSPLIT == 1 || C::ROWS, "channel groups need the row-reuse path");
        u32x4_t af[NJW];
#pragma unroll
        for (int j = 0; j < NJW; ++j) af[j] = C::WLDS ? lw[(ch * NJW + j) * 64 + lane]
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
              for (int q = 0; q < 4; ++q) bfr[r][q] = pk_bf16(vals[2 * q], vals[2 * q + 1]);
            } else {
#pragma unroll
              for (int q = 0; q < 4; ++q) bfr[r][q] = f2u(vals[q]);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
          for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], af[j], bfr[r]);
      }
    }
    // ---- epilogue ----------------------------------------------------------------
    if constexpr (PIPE) {
      // pieces of the previous tile that found no matrix-core group to hide in
#pragma unroll
      for (int k = 9 * C::CPT; k < NPIECE; ++k) piece_prev(k);
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < NJW; ++j) {
          accp[r][j] = acc[r][j];
          epp.v[r][j] = ep.v[r][j];
        }
      pty0 = ty0;
      ptx0 = tx0;
      {
        const int rows = a.H - ty0 < TH ? a.H - ty0 : TH;
        const size_t row0 = (static_cast<size_t>(ni) * a.H + ty0) * a.W * CO;
        prs = out_rsrc(static_cast<char*>(a.out0) + row0 * C::GES,
                       static_cast<unsigned>(rows) * a.W * CO * C::GES);
      }
    } else {
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < NJW; ++j)
          epilogue_piece<C, CO, EPI>(a, acc[r][j], ep.v[r][j], bias_r[j], ni, ty0, tx0, wv, r,
                                     jh * NJW + j, g, c16, sp);
    }
  };

  if constexpr (DEPTH == 1) {
    while (t < ntiles) {
      const int tn = next_open(t);
      tile(pf, t, tn);
      t = tn;
    }
  } else {
    // tiles alternate between the two buffers: t staged from pf (refilled with
    // the tile after t1), t1 from pf2
    while (t < ntiles) {
      int t2 = next_open(t1);
      tile(pf, t, t2);
      t = t1;
      t1 = t2;
      if (t >= ntiles) break;
      t2 = next_open(t1);
      tile(pf2, t, t2);
      t = t1;
      t1 = t2;
    }
  }
  if constexpr (PIPE) {
#pragma unroll
    for (int k = 0; k < NPIECE; ++k) piece_prev(k);
  }
}

template <int PREC, int CI, int CO, int PRO, int EPI>
int launch_shape(const ConvArgs& a, hipStream_t s) {
  using C = Cfg<PREC, CI, CO, PRO>;
  static_assert(C::LDS <= 160 * 1024, "LDS budget");
  static_assert(CO > 4 || EPI == E_RES || EPI == E_SUB || EPI == E_ADD,
                "thin outputs are NCHW state tensors");
  static bool attr_set = false;
  static int max_blocks = 0;
  auto kern = conv_mfma_kernel<PREC, CI, CO, PRO, EPI>;
  if (!attr_set) {
    IDQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS));
    int dev = 0, ncu = 0, occ = 0;
    IDQ_HIP(hipGetDevice(&dev));
    IDQ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    IDQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, C::THREADS, C::LDS));
    if (occ < 1) return fail(IDQ_E_UNSUPPORTED, "MFMA conv does not fit on a compute unit");
    max_blocks = ncu * occ;
    attr_set = true;
  }
  const int ntx = (a.W + TW - 1) / TW, nty = (a.H + TH - 1) / TH;
  // the pipelined epilogue addresses one tile's rows through a buffer resource
  // whose byte count must stay below the drop offset
  if (static_cast<long long>(TH) * a.W * CO * 4 >= static_cast<long long>(kDropOffset))
    return fail(IDQ_E_UNSUPPORTED, "image too wide for the MFMA conv");
  const long long nt = static_cast<long long>(a.NI) * ntx * nty;
  if (nt > 0x7fffffff) return fail(IDQ_E_INVAL, "too many tiles");
  const int ntiles = static_cast<int>(nt);
  // tile walkers (each CSPLIT workgroups, one per channel group), all resident
  const int walkers_max = max_blocks / C::CSPLIT > 0 ? max_blocks / C::CSPLIT : 1;
  const int grid = (ntiles < walkers_max ? ntiles : walkers_max) * C::CSPLIT;
  if (a.ev0) {
    ConvArgs ac = a;
    int nx = ntx, ny = nty, ntl = ntiles;
    void* args[] = {&ac, &nx, &ny, &ntl};
    IDQ_HIP(hipExtLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                               dim3(C::THREADS), args, C::LDS, s, a.ev0, a.ev1, 0));
  } else {
    kern<<<grid, C::THREADS, C::LDS, s>>>(a, ntx, nty, ntiles);
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

// (CI, CO) pairs with an MFMA instantiation: the 3->64->...->64->3 and
// 1->16->16->1 regularizers, the warm-start encoder-decoder, and their
// transposes.  Image-facing outputs (CO <= 4) are NCHW state tensors.
#define IDQ_MFMA_WIDE(X) \
  X(1, 16) X(16, 16) X(3, 64) X(64, 64) X(3, 32) X(32, 32) X(32, 64) X(64, 32) X(96, 32) X(32, 96)
#define IDQ_MFMA_THIN(X) X(16, 1) X(64, 3) X(32, 3)
// split (hi/lo bf16) instantiations: the channel counts that are whole K chunks
// (image-facing outputs run in float32 on the vector ALUs, k_conv_thin.hip)
#define IDQ_MFMA_SPLIT(X) X(64, 64) X(32, 32) X(32, 64) X(64, 32) X(64, 3)

}  // namespace mfma
}  // namespace idq
