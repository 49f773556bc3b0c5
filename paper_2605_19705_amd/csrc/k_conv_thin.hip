// Conv passes with an image-facing output: CI in {16, 32, 64} NHWC activation
// channels to CO in {1, 3} NCHW state channels (the last layer of N_theta,
// the transpose of its first layer, the warm start's output layer; eq. GS).
//
// A 3-channel output leaves 13 of 16 matrix-core columns empty, and the pass
// is bound by the activation read (CI floats per pixel), so it runs on the
// vector ALUs in float32 instead:
//   * a group of CI/4 lanes shares one output pixel, each lane holding 4 input
//     channels, so one 16-byte load per lane makes the wave read whole pixels
//     (4 pixels x 256 bytes when CI = 64) contiguously;
//   * the weights sit in LDS as one float4 (4 channels) per (tap, lane group,
//     output), so a lane reads CO 16-byte words per tap;
//   * a lane covers R rows of one column: it loads R + 2 rows per column
//     offset dx once and uses them for the three dy taps;
//   * loads are buffer loads without branches: padding offsets fall outside
//     the resource and read zero;
//   * the group's partial sums meet in its last lane through DPP row shifts
//     (no LDS), which then applies the epilogue and stores.
// Float32 passes only (the split-bf16 phase runs these layers in float32 too);
// bf16 passes stay on the matrix cores, which read half the bytes.
//
// Measured on the 8 x 3 x 256 x 256 batch: ~50 us per 64 -> 3 pass, against
// 103 us for the float32 and 67 us for the split-bf16 matrix-core forms.  Each
// item's loads are issued together and the other waves of the SIMD cover their
// latency (a software-pipelined walk with two items in flight measured slower:
// its registers halve the waves per SIMD).
#include "kernels.h"

namespace idq {

namespace {

constexpr int kThinThreads = 256;  // 4 waves
constexpr int kThinRows = 4;       // output rows per lane
constexpr int kThinWaves = 4;      // waves per SIMD the register budget allows
constexpr unsigned kDrop = 0x80000000u;  // buffer offset beyond every resource: loads 0

// Buffer resource over `bytes` at `base` (wave-uniform arguments).
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, unsigned bytes) {
  const uint64_t p = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(p));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(p >> 32));
  return __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo), static_cast<short>(0),
      static_cast<int>(__builtin_amdgcn_readfirstlane(bytes)), 0x00020000);
}

typedef __attribute__((ext_vector_type(4))) unsigned u32x4_v;

// 4 channels of one pixel as loaded (16 bytes)
struct Quad {
  u32x4_v u;
  __device__ void load(__amdgpu_buffer_rsrc_t rs, unsigned off) {
    u = __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(off), 0, 0);
  }
  __device__ float4 f() const {
    return make_float4(__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z),
                       __uint_as_float(u.w));
  }
};

// v + v(lane - n) within each row of 16 lanes (lanes below n add 0)
template <int N>
__device__ inline float add_row_shr(float v) {
  const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + N, 0xf, 0xf, true);
  return v + __int_as_float(s);
}

// One wave's operands for an item (R rows x PPW columns of one image): the
// R + 2 input rows at the three column offsets, and the epilogue operand.
template <int CO>
struct ThinItem {
  Quad v[3][kThinRows + 2];
  float e[kThinRows][CO];
};

template <int CI, int CO, int EPI>
__global__ __launch_bounds__(kThinThreads, kThinWaves) void conv_thin_kernel(ConvArgs a, int nsx, int nsy,
                                                                    int nitems) {
  constexpr int G = CI / 4;       // lanes per pixel
  constexpr int PPW = 64 / G;     // pixels (columns) per wave
  constexpr int R = kThinRows;
  static_assert(CI % 4 == 0 && G <= 16 && 16 % G == 0, "lane groups must tile a DPP row");
  const int lane = threadIdx.x & 63;
  const int cg = lane % G, col = lane / G;
  // wave-uniform: the item walk and its index arithmetic stay on the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (kThinThreads / 64) +
                                                  (threadIdx.x >> 6));
  const int nwaves = gridDim.x * (kThinThreads / 64);
  const float* in = static_cast<const float*>(a.in0);
  const float* wg = static_cast<const float*>(a.wgt);   // [CO][CI][9]
  const float* e0 = static_cast<const float*>(a.e0);
  float* out = static_cast<float*>(a.out0);
  const int H = a.H, W = a.W;
  const unsigned in_bytes = static_cast<unsigned>(H * W * CI * sizeof(float));
  const unsigned st_bytes = static_cast<unsigned>(CO * H * W * 4);
  float bias[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) bias[co] = a.bias ? static_cast<const float*>(a.bias)[co] : 0.f;

  // weights: lw[(t * G + group) * CO + co] = W[co][4 group .. 4 group + 3][t]
  __shared__ float4 lw[9 * G * CO];
  for (int i = threadIdx.x; i < 9 * G * CO; i += kThinThreads) {
    const int co = i % CO, grp = (i / CO) % G, t = i / (CO * G);
    const float* p = wg + (co * CI + 4 * grp) * 9 + t;
    lw[i] = make_float4(p[0], p[9], p[18], p[27]);
  }
  __syncthreads();

  auto open = [&](int it) {
    return gate_open_uniform(a.gate, a.gate_mask, (it / (nsx * nsy)) / a.img_div);
  };
  auto next_open = [&](int it) {
    while (it < nitems && !open(it)) it += nwaves;
    return it;
  };
  // issue the loads of item `it` (none past the last item: every offset drops).
  // Zero padding comes from the resource bounds: a row above the image has a
  // negative offset (beyond the range as unsigned), a row below it starts past
  // the end; only columns outside the image need the drop offset.
  const unsigned row_bytes = static_cast<unsigned>(W * CI * sizeof(float));
  auto fetch = [&](ThinItem<CO>& d, int it) {
    const bool live = it < nitems;
    const int itc = live ? it : 0;
    const int sx = itc % nsx, rest = itc / nsx, sy = rest % nsy, ni = rest / nsy;
    const __amdgpu_buffer_rsrc_t ri = rsrc(in + static_cast<size_t>(ni) * H * W * CI, in_bytes);
    const __amdgpu_buffer_rsrc_t re = rsrc(e0 + static_cast<size_t>(ni) * CO * H * W, st_bytes);
    const int x = sx * PPW + col, y0 = sy * R;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int xx = x + dx - 1;
      const unsigned o0 = (live && xx >= 0 && xx < W)
                              ? static_cast<unsigned>(((y0 - 1) * W + xx) * CI + 4 * cg) *
                                    static_cast<unsigned>(sizeof(float))
                              : kDrop;
#pragma unroll
      for (int r = 0; r < R + 2; ++r) d.v[dx][r].load(ri, o0 + r * row_bytes);
    }
    // every lane of a pixel's group reads the same words (one access per wave)
    const unsigned e_off = live ? static_cast<unsigned>(y0 * W + x) * 4u : kDrop;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int co = 0; co < CO; ++co)
        d.e[r][co] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
            re, static_cast<int>(e_off + static_cast<unsigned>((co * H + r) * W) * 4u), 0, 0));
  };
  unsigned long long done_px = 0;  // pixels this wave computed (lane 0)
  auto compute = [&](const ThinItem<CO>& d, int it) {
    // the weight reads below are the same for every item: keep the compiler
    // from hoisting all 9 x CO of them into registers for the whole walk
    __asm__ volatile("" ::: "memory");
    const int sx = it % nsx, rest = it / nsx, sy = rest % nsy, ni = rest / nsy;
    const int x = sx * PPW + col, y0 = sy * R;
    float acc[R][CO];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int co = 0; co < CO; ++co) acc[r][co] = 0.f;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      float4 f[R + 2];
#pragma unroll
      for (int r = 0; r < R + 2; ++r) f[r] = d.v[dx][r].f();
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        float4 wt[CO];
#pragma unroll
        for (int co = 0; co < CO; ++co) wt[co] = lw[((dy * 3 + dx) * G + cg) * CO + co];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int co = 0; co < CO; ++co) {
            float s = acc[r][co];
            s = fmaf(wt[co].x, f[r + dy].x, s);
            s = fmaf(wt[co].y, f[r + dy].y, s);
            s = fmaf(wt[co].z, f[r + dy].z, s);
            s = fmaf(wt[co].w, f[r + dy].w, s);
            acc[r][co] = s;
          }
      }
    }
    // sum over the G lanes of the pixel: it ends in lane G - 1 of the group
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int co = 0; co < CO; ++co) {
        float s = acc[r][co];
        if (G > 1) s = add_row_shr<1>(s);
        if (G > 2) s = add_row_shr<2>(s);
        if (G > 4) s = add_row_shr<4>(s);
        if (G > 8) s = add_row_shr<8>(s);
        acc[r][co] = s;
      }
    if (cg == G - 1 && x < W) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (y0 + r >= H) break;
#pragma unroll
        for (int co = 0; co < CO; ++co) {
          const size_t o = ((static_cast<size_t>(ni) * CO + co) * H + y0 + r) * W + x;
          float res;
          if (EPI == E_RES)
            res = d.e[r][co] - (acc[r][co] + bias[co]);
          else if (EPI == E_SUB)
            res = d.e[r][co] - acc[r][co];
          else
            res = d.e[r][co] + (acc[r][co] + bias[co]);
          out[o] = res;
        }
      }
    }
    if (a.work_px && lane == 0) {
      const int cols = W - sx * PPW < PPW ? W - sx * PPW : PPW;
      const int rows = H - y0 < R ? H - y0 : R;
      done_px += static_cast<unsigned long long>(rows * cols);
    }
  };

  // all of an item's loads are issued together; the other waves of the SIMD
  // cover their latency
  ThinItem<CO> A;
  for (int item = next_open(wave); item < nitems; item = next_open(item + nwaves)) {
    fetch(A, item);
    compute(A, item);
  }
  // one counter update per wave (one per item would serialise on the address)
  if (a.work_px && lane == 0 && done_px) atomicAdd(a.work_px, done_px);
}

template <int CI, int CO, int EPI>
int launch_thin(const ConvArgs& a, hipStream_t s) {
  constexpr int PPW = 64 / (CI / 4);
  auto kern = conv_thin_kernel<CI, CO, EPI>;
  static int max_blocks = 0;
  if (max_blocks == 0) {
    int dev = 0, ncu = 0, occ = 0;
    IDQ_HIP(hipGetDevice(&dev));
    IDQ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    IDQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kThinThreads, 0));
    if (occ > 4) occ = 4;
    if (occ < 1) return fail(IDQ_E_UNSUPPORTED, "thin conv does not fit on a compute unit");
    max_blocks = ncu * occ;
  }
  const long long nsx = (a.W + PPW - 1) / PPW, nsy = (a.H + kThinRows - 1) / kThinRows;
  // per-image byte offsets are 32-bit: the image (plus the rows an item reads
  // past a dropped or negative start) must stay below the drop offset
  const long long span = static_cast<long long>(a.H + kThinRows + 2) * a.W;
  if (span * CI * static_cast<long long>(sizeof(float)) >= static_cast<long long>(kDrop) / 2 ||
      span * CO * 4 >= static_cast<long long>(kDrop) / 2)
    return fail(IDQ_E_UNSUPPORTED, "image too large for the thin conv");
  const long long items = static_cast<long long>(a.NI) * nsx * nsy;
  if (items > 0x7fffffff) return fail(IDQ_E_INVAL, "too many pixels in one conv pass");
  const int nitems = static_cast<int>(items);
  const long long want = (items + 3) / 4;
  const int grid = static_cast<int>(want < max_blocks ? want : max_blocks);
  int ix = static_cast<int>(nsx), iy = static_cast<int>(nsy);
  if (a.ev0) {
    ConvArgs ac = a;
    void* args[] = {&ac, &ix, &iy, const_cast<int*>(&nitems)};
    IDQ_HIP(hipExtLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                               dim3(kThinThreads), args, 0, s, a.ev0, a.ev1, 0));
  } else {
    kern<<<grid, kThinThreads, 0, s>>>(a, ix, iy, nitems);
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

template <int CI, int CO>
int by_epi(const ConvArgs& a, hipStream_t s) {
  switch (a.epi) {
    case E_RES: return launch_thin<CI, CO, E_RES>(a, s);
    case E_SUB: return launch_thin<CI, CO, E_SUB>(a, s);
    case E_ADD: return launch_thin<CI, CO, E_ADD>(a, s);
    default: return fail(IDQ_E_UNSUPPORTED, "thin conv epilogue");
  }
}

int by_shape(const ConvArgs& a, hipStream_t s) {
  if (a.CI == 64 && a.CO == 3) return by_epi<64, 3>(a, s);
  if (a.CI == 32 && a.CO == 3) return by_epi<32, 3>(a, s);
  if (a.CI == 16 && a.CO == 1) return by_epi<16, 1>(a, s);
  return fail(IDQ_E_UNSUPPORTED, "thin conv shape");
}

}  // namespace

bool thin_supported(const ConvArgs& a, int prec) {
  const bool shape = (a.CI == 64 && a.CO == 3) || (a.CI == 32 && a.CO == 3) ||
                     (a.CI == 16 && a.CO == 1);
  // bf16 passes stay on the matrix cores, which read half the bytes as fast
  return shape && prec == PREC_F32 && a.in_fmt == F_NHWC &&
         a.out_fmt == F_NCHW && a.pro == P_NONE &&
         (a.epi == E_RES || a.epi == E_SUB || a.epi == E_ADD) && a.wgt != nullptr;
}

int launch_conv_thin(const ConvArgs& a, int prec, hipStream_t s) {
  if (!thin_supported(a, prec)) return fail(IDQ_E_UNSUPPORTED, "thin conv pass of an unsupported form");
  return by_shape(a, s);
}

}  // namespace idq
