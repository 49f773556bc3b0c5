// 3x3 convolutions from 64 input channels (to 32 or 64 activation channels, or
// in split-bf16 to 3 NCHW state channels) in split-bf16, bf16 or float32
// arithmetic, software-pipelined over the two halves of the input channels,
// with the halo traffic on waves of its own.
//
// Same arithmetic as conv_mfma_kernel (k_conv_mfma.h).  Split: float
// activations and float weights each taken as a bf16 hi part plus the bf16
// rounding of the remainder, acc += W_lo x_hi + W_hi x_lo + W_hi x_hi on
// v_mfma_f32_16x16x32_bf16.  Bf16: bf16 activations, one product.  Float32:
// v_mfma_f32_16x16x4f32 on float4 slices of 16-channel K chunks.  Split and
// float32 take 32 output channels per workgroup (two workgroups per tile for
// 64 outputs, on one XCD) so that the weight fragments (split: hi and lo) fit
// in LDS beside the 18 x 18 halo tile (161,856 bytes: one workgroup per
// compute unit); bf16 takes all 64, and a 3-channel output one block of 16
// matrix rows.
//
// What differs is the schedule.  The K loop runs channel half 0 (K chunks of
// input channels 0..31, all 9 taps) and then channel half 1.  Each half reads
// only its own bytes of every halo pixel, so while half 0 of tile t is on the
// matrix cores, half 1 of the same tile goes from registers into LDS, and
// while half 1 is, half 0 of the next tile does: the LDS footprint stays that
// of one tile.  The workgroup's 8 waves split the work: waves 0..3 (one per
// SIMD, 4 output rows each) run the K loop and the epilogue; waves 4..7 load
// the halo from HBM one half ahead, split it into hi and lo parts (split
// arithmetic) and write it to LDS.  A vector memory instruction in a wave that
// feeds the matrix core holds up its MFMA stream; on the helper waves it only
// occupies the SIMD's issue slots the MFMA wave leaves free.  The epilogue
// (SoftPlus or sigma', stores) of a tile follows its K loop.  Per matrix wave
// and (dx, chunk) step the six input rows are read once for the three kernel
// rows (dy) that use them, a third of them per group during the previous
// step; weight fragment reads are issued one matrix-core group ahead;
// scheduling-group hints spread the reads between the MFMAs.  Both kinds of
// wave walk the same tiles and meet at the same two barriers per tile, in
// loops of their own (so that their registers are not live at once).
#pragma once

#include "k_conv_mfma.h"

namespace idq {
namespace mfma {

constexpr int kS64Threads = 512;  // 4 matrix waves, then 4 halo waves

template <int PREC, int CO, int EPI>
__global__ __launch_bounds__(kS64Threads, 1) void conv_halves_kernel(ConvArgs a, int ntx,
                                                                     int nty, int ntiles) {
  using C = Cfg<PREC, 64, CO, P_NONE>;
  constexpr bool SPLIT = PREC == PREC_SPLIT, BF = PREC == PREC_BF16;
  static_assert(SPLIT || BF || PREC == PREC_F32, "split-bf16, bf16 or float32 arithmetic");
  // THIN: an image-facing output (CO <= 4 NCHW state channels, one block of 16
  // matrix rows of which CO are used)
  constexpr bool THIN = CO <= 4;
  static_assert((THIN ? C::NJW == 1 : (C::NJW == 2 || C::NJW == 4)) && TW == 16 && C::WLDS &&
                    (!SPLIT || C::WLO_LDS) &&
                    (SPLIT ? (C::CPT == 2 && C::LO_OFF == 128) : C::CPT == (BF ? 2 : 4)),
                "shape of the channel-half pipeline");
  static_assert(THIN ? (EPI == E_RES || EPI == E_SUB)
                     : (EPI == E_ACT || EPI == E_DELTA || EPI == E_RAW),
                "NHWC activation outputs, or NCHW state outputs for CO <= 4");
  constexpr int NT_ = kS64Threads / 2, RW = TH / (NT_ / 64), NJW = C::NJW, NR = RW + 2;
  // K chunks of one half per tap (split and bf16: 32 channels; float32: 2 x
  // 16), the LDS bytes of a channel quad (float32 in HBM) and of a half within
  // a halo pixel, and the bytes of an activation in HBM
  constexpr int CPH = C::CPT / 2;
  constexpr int QB = SPLIT ? 8 : 16, HB = SPLIT || BF ? 64 : 128, EB = BF ? 2 : 4;

  // 16-byte items of one channel half (4 float or 8 bf16 channels of one
  // pixel), per thread
  constexpr int HITEMS = NPIX * (BF ? 4 : 8);
  constexpr int NHI = (HITEMS + NT_ - 1) / NT_;
  static_assert(RW % 2 == 0, "sigma(h) is read in two groups");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  char* lin = smem;
  const u32x4_t* lw = reinterpret_cast<const u32x4_t*>(smem + C::LDS_IN);
  const u32x4_t* lwl = lw + C::NCH * NJW * 64;
  const u32x4_t* gw = static_cast<const u32x4_t*>(a.wmfma);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, g = lane >> 4, c16 = lane & 15;
  const bool sp = a.act == IDQ_ACT_SOFTPLUS;
  const int tiles_per_img = ntx * nty;
  auto open = [&](int tt) {
    return gate_open_uniform(a.gate, a.gate_mask, (tt / tiles_per_img) / a.img_div);
  };

  // channel group and tile walk (as in conv_mfma_kernel)
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
  int t = walker;
  while (t < ntiles && !open(t)) t += tstep;
  if (t >= ntiles) return;
  auto next_open = [&](int tt) {
    tt += tstep;
    while (tt < ntiles && !open(tt)) tt += tstep;
    return tt;
  };

  // Items of a half, float activations (16 bytes: 4 channels of one halo
  // pixel; bf16 activations: 8 channels, item i of the tile is quarter i % 4 of
  // the half of pixel i / 4, copied as loaded).  Items 0..8 of
  // a thread walk the 16 inner columns two rows at a time: row 2k + tid / 128,
  // column 1 + (tid / 8) % 16, channel quad tid % 8, so that one item's offset
  // is the thread's offset plus a uniform step.  Items 9 and 10 cover the two
  // edge columns (288 items: e = tid + 256 (k - 9), row e / 16, column 0 or 17
  // by bit 3 of e, quad e % 8).  Loads go through a buffer resource over the
  // tile's image: 32-bit offsets, and an offset outside the image (a halo row
  // above or below it, or an offset pushed past it for a column outside it)
  // reads zero.  Branch-free, so that it can be scheduled among the MFMAs:
  // past the last tile the resource covers zero bytes.
  static_assert(NT_ == 256 && TW == 16 && NHI == (BF ? 6 : 11), "halo item layout");
  const unsigned img_bytes = static_cast<unsigned>(a.H * a.W) * (64u * EB);
  const int htid = tid & (NT_ - 1);  // thread index among the halo waves
  // inner column of this thread's items: 8-lane groups take columns in the
  // order 0, 4, 1, 5, 2, 6, 3, 7, 8, 12, ..., so that the two groups of 16
  // lanes an LDS write serves together hit different banks (4 pixels apart)
  const int jcol = (htid >> 3) & 15;
  const int col_i = 1 + ((jcol & 1) << 2) + ((jcol >> 1) & 3) + (jcol & 8), q_i = htid & 7,
            r0 = htid >> 7;
  const int thr_int = (r0 * a.W + col_i) * 256 + q_i * 16;
  const int lds_int = ((r0 * HW_ + col_i) * C::PIXB) + q_i * QB;
  int e_row[2], e_col[2], thr_e[2], lds_e[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int e = htid + 256 * m;
    e_row[m] = e >> 4;
    e_col[m] = ((e >> 3) & 1) ? HW_ - 1 : 0;
    thr_e[m] = (e_row[m] * a.W + e_col[m]) * 256 + (e & 7) * 16;
    lds_e[m] = (e_row[m] * HW_ + e_col[m]) * C::PIXB + (e & 7) * QB;
  }
  auto load_half = [&](u32x4_t (&buf)[NHI], int tt, int h, int k0, int k1) {
    const bool real = tt < ntiles;
    const int tc = real ? tt : 0;
    const int ni = tc / tiles_per_img, rem = tc - ni * tiles_per_img;
    const int ty0 = (rem / ntx) * TH, tx0 = (rem % ntx) * TW;
    const __amdgpu_buffer_rsrc_t rs = out_rsrc(
        const_cast<char*>(static_cast<const char*>(a.in0)) + static_cast<size_t>(ni) * img_bytes,
        real ? img_bytes : 0u);
    // byte offset of halo pixel (0, 0) of this tile and half, float
    // activations (negative on the top row of images: those rows read zero)
    const int org = ((ty0 - 1) * a.W + tx0 - 1) * 256 + h * 128;
    const int base_i = tx0 - 1 + col_i < a.W ? thr_int : static_cast<int>(kDropOffset);
#pragma unroll
    for (int k = k0; k < k1; ++k) {
      int off;
      if constexpr (BF) {
        // bf16: item it = htid + 256 k is pixel it / 4, channels 32 h + 8 (it % 4) .. + 7
        const int it = htid + k * NT_, p = it >> 2, q = it & 3;
        const int ly = p / HW_, lx = p - (p / HW_) * HW_;
        const int gy = ty0 - 1 + ly, gx = tx0 - 1 + lx;
        const bool in = it < HITEMS && static_cast<unsigned>(gy) < static_cast<unsigned>(a.H) &&
                        static_cast<unsigned>(gx) < static_cast<unsigned>(a.W);
        off = in ? (gy * a.W + gx) * 128 + h * 64 + q * 16 : static_cast<int>(kDropOffset);
      } else if (k < 9) {
        off = base_i + (org + k * 2 * a.W * 256);
      } else {
        const int m = k - 9;
        const bool ok = e_col[m] == 0 ? tx0 > 0 : tx0 + HW_ - 2 < a.W;
        off = ok && htid + 256 * m < HITEMS ? thr_e[m] + org : static_cast<int>(kDropOffset);
      }
      const u32x4_v v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
      buf[k] = u32x4_t{v[0], v[1], v[2], v[3]};
    }
  };
  // item k into the half's LDS bytes: split, the hi parts and the
  // bf16-rounded remainders; float32, the values
  auto store_item = [&](const u32x4_t (&buf)[NHI], int k, int h) {
    if constexpr (BF) {
      const int it = htid + k * NT_;
      if ((k + 1) * NT_ <= HITEMS || it < HITEMS)
        *reinterpret_cast<u32x4_t*>(lin + (it >> 2) * C::PIXB + h * HB + (it & 3) * 16) = buf[k];
      return;
    }
    // items 0..9 exist for every thread, item 10 for the first 32
    if (k < 10 || htid < HITEMS - 10 * NT_) {
      const u32x4_t val = buf[k];
      char* d = lin + h * HB + (k < 9 ? lds_int + k * 2 * HW_ * C::PIXB : lds_e[k < 9 ? 0 : k - 9]);
      if constexpr (SPLIT) {
        const unsigned h01 = pk_bf16(u2f(val[0]), u2f(val[1]));
        const unsigned h23 = pk_bf16(u2f(val[2]), u2f(val[3]));
        const unsigned l01 = pk_bf16(u2f(val[0]) - u2f(h01 << 16), u2f(val[1]) - u2f(h01 & 0xffff0000u));
        const unsigned l23 = pk_bf16(u2f(val[2]) - u2f(h23 << 16), u2f(val[3]) - u2f(h23 & 0xffff0000u));
        *reinterpret_cast<uint2*>(d) = uint2{h01, h23};
        *reinterpret_cast<uint2*>(d + C::LO_OFF) = uint2{l01, l23};
      } else {
        *reinterpret_cast<u32x4_t*>(d) = val;
      }
    }
  };

  const bool halo_wave = tid >= NT_;
  u32x4_t b0[NHI], b1[NHI];
  if (halo_wave) {
    load_half(b0, t, 0, 0, NHI);
    load_half(b1, t, 1, 0, NHI);
  }
  {
    // this workgroup's hi and lo weight fragments into LDS, in fragment order
    constexpr int NW = C::NCH * NJW * 64;
    constexpr int NT = (SPLIT ? 2 : 1) * NW;  // hi and lo fragments for split
    constexpr int PER = (NT + kS64Threads - 1) / kS64Threads;
    constexpr int WB = PER < 24 ? PER : 24;
    u32x4_t* dst = reinterpret_cast<u32x4_t*>(smem + C::LDS_IN);
    auto src = [&](int i) {
      const int part = i >= NW ? 1 : 0, f = i - part * NW;
      const int ln = f % 64, jj = (f / 64) % NJW, ch = f / (64 * NJW);
      return (part * C::NCH * C::NJ + ch * C::NJ + jh * NJW + jj) * 64 + ln;
    };
    for (int q0 = 0; q0 < PER; q0 += WB) {
      u32x4_t wbuf[WB];
#pragma unroll
      for (int q = 0; q < WB; ++q) {
        const int i = tid + (q0 + q) * kS64Threads;
        if (i < NT) wbuf[q] = gw[src(i)];
      }
#pragma unroll
      for (int q = 0; q < WB; ++q) {
        const int i = tid + (q0 + q) * kS64Threads;
        if (i < NT) dst[i] = wbuf[q];
      }
    }
  }
  // this workgroup's 16 NJW biases, after the weights (read by the epilogue)
  float* lbias = reinterpret_cast<float*>(smem + C::LDS);
  if (tid < 16 * NJW) {
    const float* bias = static_cast<const float*>(a.bias);
    const int co = 16 * jh * NJW + tid;
    lbias[tid] = (bias && co < CO) ? bias[co] : 0.f;
  }
  if (halo_wave) {
#pragma unroll
    for (int k = 0; k < NHI; ++k) store_item(b0, k, 0);
  }
  __syncthreads();  // the first tile's half 0, the weights and biases are in LDS

  if (halo_wave) {
    // Halo waves.  Half 0 of tile t: t's half 1 (b1) into LDS, then b0 takes
    // the next tile's half 0.  Half 1: that into LDS (past the last tile b0
    // holds zeros, stored to no effect), then b1 takes the next tile's half 1.
    // Each half waits once, for loads issued a half earlier.
    while (t < ntiles) {
      const int tn = next_open(t);
#pragma unroll
      for (int k = 0; k < NHI; ++k) store_item(b1, k, 1);
      load_half(b0, tn, 0, 0, NHI);
      __syncthreads();  // half 1 of t is in LDS; the matrix waves are done with half 0
#pragma unroll
      for (int k = 0; k < NHI; ++k) store_item(b0, k, 0);
      load_half(b1, tn, 1, 0, NHI);
      __syncthreads();  // half 0 of tn is in LDS; the matrix waves are done with half 1
      t = tn;
    }
    return;
  }

  // the tile's sigma(h) operand (E_DELTA): 4 channels per piece, as floats or
  // packed bf16; for THIN outputs the state operand e0 of the CO channels
  constexpr int EW = BF ? 2 : 4;
  unsigned e0v[RW][NJW][EW];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int j = 0; j < NJW; ++j)
#pragma unroll
      for (int i = 0; i < EW; ++i) e0v[r][j][i] = 0u;
  // the output resource over the tile's rows, and the lane part of a piece's
  // byte offset in them (past the image's right edge: pushed beyond the
  // resource)
  __amdgpu_buffer_rsrc_t prs = out_rsrc(a.out0, 0u);
  const int wvu = __builtin_amdgcn_readfirstlane(wv);
  int plane = static_cast<int>(kDropOffset);
  // THIN: rows of the tile inside the image
  int rows_in = 0;
  auto piece = [&](int r, int jj, const f32x4_t& accv) {
    const int ly = wvu * RW + r;
    if constexpr (THIN) {
      // lanes 0..15 hold output channels 0..3 of pixel c16 (channels >= CO are
      // padding); NCHW planes of the tile's image, rows past its bottom dropped
      const bool ok = ly < rows_in && plane != static_cast<int>(kDropOffset);
#pragma unroll
      for (int i = 0; i < CO; ++i) {
        const float x = accv[i];
        const float e = u2f(e0v[r][0][i]);
        const float v = EPI == E_RES ? e - (x + lbias[i]) : e - x;
        const int off = ok ? plane + (ly * a.W + i * a.H * a.W) * 4 : static_cast<int>(kDropOffset);
        __builtin_amdgcn_raw_buffer_store_b32(f2u(v), prs, off, 0, 0);
      }
      return;
    }
    float v[4];
    float4 bias4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (EPI == E_ACT) bias4 = *reinterpret_cast<const float4*>(lbias + 16 * jj + 4 * g);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float x = accv[i];
      // both forms computed and selected (no branch among the MFMAs)
      if constexpr (EPI == E_ACT) {
        const float hv = x + (i == 0 ? bias4.x : i == 1 ? bias4.y : i == 2 ? bias4.z : bias4.w);
        const float y = BF ? softplus_fast(hv) : softplus_hw(hv);
        v[i] = sp ? y : hv;
      } else if constexpr (EPI == E_DELTA) {
        const float av = BF ? u2f((e0v[r][jj][i >> 1] << ((i & 1) ? 0 : 16)) & 0xffff0000u)
                            : u2f(e0v[r][jj][i]);
        const float d = BF ? dsp_from_a_fast(av) : dsp_from_a_hw(av);
        v[i] = (sp ? d : 1.f) * x;
      } else {
        v[i] = x;
      }
    }
    // rows past the image's bottom edge fall outside the resource
    const int off = plane + (ly * a.W * CO * EB + jj * 16 * EB);
    if constexpr (BF) {
      const u32x2_v pk = {pk_bf16(v[0], v[1]), pk_bf16(v[2], v[3])};
      __builtin_amdgcn_raw_buffer_store_b64(pk, prs, off, 0, 0);
    } else {
      const u32x4_v pk = {f2u(v[0]), f2u(v[1]), f2u(v[2]), f2u(v[3])};
      __builtin_amdgcn_raw_buffer_store_b128(pk, prs, off, 0, 0);
    }
  };

  // LDS bases of this lane's row and weight reads: every read is one of them
  // plus an immediate offset below 64 KB (left to itself the compiler keeps an
  // address register per row and weight block, some 90 VGPRs)
  const char* rbase = lin + ((wvu * RW * HW_ + c16) * C::PIXB + g * 16);
  const u32x4_t* whb = lw + lane;
  const u32x4_t* wlb = lwl + lane;
  while (t < ntiles) {
    const int tn = next_open(t);
    const int ni = t / tiles_per_img;
    const int rem = t - ni * tiles_per_img;
    const int ty0 = (rem / ntx) * TH, tx0 = (rem % ntx) * TW;
    if (a.work_px && tid == 0 && jh == 0) {
      const int vh = a.H - ty0 < TH ? a.H - ty0 : TH, vw = a.W - tx0 < TW ? a.W - tx0 : TW;
      atomicAdd(a.work_px, static_cast<unsigned long long>(vh * vw));
    }
    f32x4_t acc[RW][NJW];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int j = 0; j < NJW; ++j) acc[r][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    // one channel half of the K loop: 3 (dx) x 3 (dy) groups of 3 RW NJW MFMAs,
    // and after each group's MFMAs the side work `side(group)`
    auto half = [&](const int c, auto&& side) {
      // NS steps (dx, chunk) of three groups (dy).  Eight row slots: step st
      // holds its input row ir in slot kSlot[st % 4][ir]; a slot is refilled as
      // soon as the kernel rows (dy) of its row are done
      static_assert(RW == 4, "row slot table for 4 output rows per wave");
      constexpr int NS = 3 * CPH;
      constexpr int kSlot[4][6] = {
          {0, 1, 2, 3, 4, 5}, {6, 7, 0, 1, 2, 3}, {4, 5, 6, 7, 0, 1}, {2, 3, 4, 5, 6, 7}};
      u32x4_t rh[8], rl[SPLIT ? 8 : 1], afc[NJW], alc[NJW], afn[NJW], aln[NJW];
      auto load_row = [&](int st, int ir) {
        const int dx = st / CPH, cl = st % CPH;
        const char* b = rbase + ((ir * HW_ + dx) * C::PIXB + c * HB + cl * 64);
        rh[kSlot[st % 4][ir]] = *reinterpret_cast<const u32x4_t*>(b);
        if constexpr (SPLIT) rl[kSlot[st % 4][ir]] = *reinterpret_cast<const u32x4_t*>(b + C::LO_OFF);
      };
      auto load_w = [&](u32x4_t* hi, u32x4_t* lo, int st, int dy) {
        const int dx = st / CPH, cl = st % CPH;
        const int ch = (dy * 3 + dx) * C::CPT + c * CPH + cl;
#pragma unroll
        for (int j = 0; j < NJW; ++j) {
          hi[j] = whb[(ch * NJW + j) * 64];
          if constexpr (SPLIT) lo[j] = wlb[(ch * NJW + j) * 64];
        }
      };
#pragma unroll
      for (int ir = 0; ir < NR; ++ir) load_row(0, ir);
      load_w(afc, alc, 0, 0);
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        const int sl = st % 4;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          // reads for later groups: rows into slots freed by earlier groups
          // (this step's rows 4 and 5 and the next step's rows 0 and 1 in group
          // 0, the next step's rows 2 and 3 in groups 1 and 2), the next
          // group's weight fragments
          if (dy == 0 && st > 0) {
            load_row(st, 4);
            load_row(st, 5);
          }
          if (st + 1 < NS) {
            if (dy == 0) {
              load_row(st + 1, 0);
              load_row(st + 1, 1);
            } else {
              load_row(st + 1, dy + 1);
            }
          }
          if (dy < 2)
            load_w(afn, aln, st, dy + 1);
          else if (st + 1 < NS)
            load_w(afn, aln, st + 1, 0);
          if constexpr (SPLIT) {
            // small terms first (lo*hi, hi*lo, then hi*hi), each term over all
            // accumulators before the next
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
              for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], afc[j], rl[kSlot[sl][r + dy]]);
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
              for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], alc[j], rh[kSlot[sl][r + dy]]);
          }
#pragma unroll
          for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int j = 0; j < NJW; ++j) mma<C>(acc[r][j], afc[j], rh[kSlot[sl][r + dy]]);
          side(st * 3 + dy);
          // spread this group's LDS reads and side work between its MFMAs
          // (split: 3 products per term; float32: 4 MFMAs per 16-channel chunk)
          constexpr int NM = (SPLIT ? 3 : BF ? 1 : 4) * RW * NJW;
#pragma unroll
          for (int i = 0; i < NM; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            if (i < 8) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // VALU
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
            __builtin_amdgcn_sched_group_barrier(0x040, 1, 0);  // VMEM write
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int j = 0; j < NJW; ++j) {
            afc[j] = afn[j];
            if constexpr (SPLIT) alc[j] = aln[j];
          }
        }
      }
    };

    // Side work of the matrix waves: this tile's sigma(h) operand (or for a
    // 3-channel output its e0 state), read in groups 5..6 of half 1 (not held
    // through the rest of it).  The epilogue follows the K loop: spreading it
    // over the next tile's half 0, with a second accumulator set, measured no
    // faster.
    half(0, [&](int) {});
    __syncthreads();  // half 1 is in LDS, half 0 has been read
    half(1, [&](int grp) {
      if (THIN && (grp == 5 || grp == 6)) {
        // this tile's e0 (z for E_RES, r for E_SUB), half of the rows per group
        const __amdgpu_buffer_rsrc_t ers =
            out_rsrc(const_cast<char*>(static_cast<const char*>(a.e0)) +
                         static_cast<size_t>(ni) * CO * a.H * a.W * 4,
                     static_cast<unsigned>(CO * a.H * a.W * 4));
        const int rows = a.H - ty0 < TH ? a.H - ty0 : TH;
        const int lane_off = g == 0 && tx0 + c16 < a.W ? (ty0 * a.W + tx0 + c16) * 4
                                                       : static_cast<int>(kDropOffset);
#pragma unroll
        for (int r = (grp - 5) * RW / 2; r < (grp - 4) * RW / 2; ++r) {
          const int ly = wvu * RW + r;
          const bool ok = ly < rows && lane_off != static_cast<int>(kDropOffset);
#pragma unroll
          for (int i = 0; i < CO; ++i) {
            const int off = ok ? lane_off + (ly * a.W + i * a.H * a.W) * 4
                               : static_cast<int>(kDropOffset);
            e0v[r][0][i] = __builtin_amdgcn_raw_buffer_load_b32(ers, off, 0, 0);
          }
        }
      }
      if (EPI == E_DELTA && (grp == 5 || grp == 6)) {
        // this tile's sigma(h) (half of it per group), through a resource over
        // its rows: pixels past the image edge read zero
        const int rows = a.H - ty0 < TH ? a.H - ty0 : TH;
        const size_t row0 = (static_cast<size_t>(ni) * a.H + ty0) * a.W * CO;
        const __amdgpu_buffer_rsrc_t ers =
            out_rsrc(const_cast<char*>(static_cast<const char*>(a.e0)) + row0 * EB,
                     static_cast<unsigned>(rows) * a.W * CO * EB);
        const int lane_off = tx0 + c16 < a.W ? ((tx0 + c16) * CO + 16 * jh * NJW + 4 * g) * EB
                                             : static_cast<int>(kDropOffset);
#pragma unroll
        for (int r = (grp - 5) * RW / 2; r < (grp - 4) * RW / 2; ++r)
#pragma unroll
          for (int jj = 0; jj < NJW; ++jj) {
            const int off = lane_off + ((wvu * RW + r) * a.W * CO * EB + jj * 16 * EB);
            if constexpr (BF) {
              const u32x2_v v = __builtin_amdgcn_raw_buffer_load_b64(ers, off, 0, 0);
              e0v[r][jj][0] = v[0];
              e0v[r][jj][1] = v[1];
            } else {
              const u32x4_v v = __builtin_amdgcn_raw_buffer_load_b128(ers, off, 0, 0);
#pragma unroll
              for (int i = 0; i < 4; ++i) e0v[r][jj][i] = v[i];
            }
          }
      }
    });
    __syncthreads();  // the next tile's half 0 is in LDS, half 1 has been read
    if constexpr (THIN) {
      // NCHW planes of the tile's image; lane part of the offset of its pixel
      // in the tile's first row
      rows_in = a.H - ty0 < TH ? a.H - ty0 : TH;
      plane = g == 0 && tx0 + c16 < a.W ? (ty0 * a.W + tx0 + c16) * 4
                                        : static_cast<int>(kDropOffset);
      prs = out_rsrc(static_cast<char*>(a.out0) + static_cast<size_t>(ni) * CO * a.H * a.W * 4,
                     static_cast<unsigned>(CO * a.H * a.W * 4));
    } else {
      plane = tx0 + c16 < a.W ? ((tx0 + c16) * CO + 16 * jh * NJW + 4 * g) * EB
                              : static_cast<int>(kDropOffset);
      const int rows = a.H - ty0 < TH ? a.H - ty0 : TH;
      const size_t row0 = (static_cast<size_t>(ni) * a.H + ty0) * a.W * CO;
      prs = out_rsrc(static_cast<char*>(a.out0) + row0 * EB, static_cast<unsigned>(rows) * a.W * CO * EB);
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int j = 0; j < NJW; ++j) piece(r, j, acc[r][j]);
    t = tn;
  }
}

// the halo loads address one image through 32-bit byte offsets
inline bool halves_fits(const ConvArgs& a) {
  // an offset pushed out of range (kDropOffset plus at most one image) must
  // stay above the image and below 2^32, one pushed below zero stay negative
  return static_cast<long long>(a.H) * a.W * 256 <= (1LL << 30) && a.W >= 16;
}

template <int PREC, int CO, int EPI>
int launch_halves(const ConvArgs& a, hipStream_t s) {
  using C = Cfg<PREC, 64, CO, P_NONE>;
  constexpr int LDS = C::LDS + 16 * C::NJW * 4;  // + this workgroup's biases
  static_assert(LDS <= 160 * 1024, "LDS budget");
  static bool attr_set = false;
  static int max_blocks = 0;
  auto kern = conv_halves_kernel<PREC, CO, EPI>;
  constexpr int THREADS = kS64Threads;
  if (!attr_set) {
    IDQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, LDS));
    int dev = 0, ncu = 0, occ = 0;
    IDQ_HIP(hipGetDevice(&dev));
    IDQ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    IDQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, THREADS, LDS));
    if (occ < 1) return fail(IDQ_E_UNSUPPORTED, "channel-half conv does not fit on a compute unit");
    max_blocks = ncu * occ;
    attr_set = true;
  }
  const int ntx = (a.W + TW - 1) / TW, nty = (a.H + TH - 1) / TH;
  if (static_cast<long long>(TH) * a.W * CO * 4 >= static_cast<long long>(kDropOffset))
    return fail(IDQ_E_UNSUPPORTED, "image too wide for the MFMA conv");
  const long long nt = static_cast<long long>(a.NI) * ntx * nty;
  if (nt > 0x7fffffff) return fail(IDQ_E_INVAL, "too many tiles");
  const int ntiles = static_cast<int>(nt);
  const int walkers_max = max_blocks / C::CSPLIT > 0 ? max_blocks / C::CSPLIT : 1;
  const int grid = (ntiles < walkers_max ? ntiles : walkers_max) * C::CSPLIT;
  if (a.ev0) {
    ConvArgs ac = a;
    int nx = ntx, ny = nty, ntl = ntiles;
    void* args[] = {&ac, &nx, &ny, &ntl};
    IDQ_HIP(hipExtLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(THREADS),
                               args, LDS, s, a.ev0, a.ev1, 0));
  } else {
    kern<<<grid, THREADS, LDS, s>>>(a, ntx, nty, ntiles);
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

}  // namespace mfma
}  // namespace idq
