// Bandwidth-bound kernels of the i-DEQ iteration: circular blur stencils of the
// forward operator, the inertial extrapolation, the fused update with its
// float64 residual partial sums, the per-image finalize step (stopping rule,
// restart, precision phase) and deterministic float64 reductions.
#include <cmath>
#include <cstdint>
#include <initializer_list>

#include "kernels.h"

namespace idq {

namespace {

constexpr int kBlock = 256;

template <typename T>
__device__ inline bool finite_v(T v) { return isfinite(v); }

// Fixed-order block reduction of up to three float64 sums (deterministic).
__device__ inline void block_sum3(double& a, double& b, double& c) {
  __shared__ double red[3][kBlock];
  const int t = threadIdx.x;
  red[0][t] = a;
  red[1][t] = b;
  red[2][t] = c;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (t < o) {
      red[0][t] += red[0][t + o];
      red[1][t] += red[1][t + o];
      red[2][t] += red[2][t + o];
    }
    __syncthreads();
  }
  a = red[0][0];
  b = red[1][0];
  c = red[2][0];
}

// ---------------------------------------------------------------------------
// Circular stencil (correlation with up to 9x9 taps) on 16x16 output tiles.
// The (16+kh-1) x (16+kw-1) input tile is staged in LDS with modular wrap.
// ---------------------------------------------------------------------------
constexpr int kTile = 16;
constexpr int kMaxTap = 9;
constexpr int kLds = (kTile + kMaxTap - 1) * (kTile + kMaxTap - 1);

template <typename T>
struct Taps {
  T k[kMaxTap * kMaxTap];
};

__device__ inline int wrap(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}
// wrap for offsets within one period of the range (the common case), without
// the integer division
__device__ inline int wrap1(int v, int n) {
  if (v < 0) v += n;
  if (v >= n) v -= n;
  return (v < 0 || v >= n) ? wrap(v, n) : v;
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void stencil_kernel(StencilArgs a, Taps<T> taps) {
  __shared__ T tile0[kLds];
  __shared__ T tile1[MODE == S_TANH_HESS ? kLds : 1];
  const int plane = blockIdx.z;
  if (a.gate && ((1 << a.gate[plane / a.plane_div]) & a.gate_mask) == 0) return;
  const int ty0 = blockIdx.y * kTile, tx0 = blockIdx.x * kTile;
  const int ry = (a.kh - 1) / 2, rx = (a.kw - 1) / 2;
  const int LH = kTile + a.kh - 1, LW = kTile + a.kw - 1;
  const size_t pbase = static_cast<size_t>(plane) * a.H * a.W;
  const T* in0 = static_cast<const T*>(a.in0) + pbase;
  const T* in1 = static_cast<const T*>(a.in1) + (MODE == S_TANH_HESS ? pbase : 0);
  for (int i = threadIdx.x; i < LH * LW; i += kBlock) {
    const int ly = i / LW, lx = i - (i / LW) * LW;
    const int gy = wrap(ty0 - ry + ly, a.H), gx = wrap(tx0 - rx + lx, a.W);
    tile0[i] = in0[static_cast<size_t>(gy) * a.W + gx];
    if (MODE == S_TANH_HESS) tile1[i] = in1[static_cast<size_t>(gy) * a.W + gx];
  }
  __syncthreads();
  const int ly = threadIdx.x / kTile, lx = threadIdx.x % kTile;
  const int oy = ty0 + ly, ox = tx0 + lx;
  if (oy >= a.H || ox >= a.W) return;
  T s0 = T(0), s1 = T(0);
  for (int p = 0; p < a.kh; ++p)
    for (int q = 0; q < a.kw; ++q) {
      const T kv = taps.k[p * a.kw + q];
      s0 += kv * tile0[(ly + p) * LW + lx + q];
      if (MODE == S_TANH_HESS) s1 += kv * tile1[(ly + p) * LW + lx + q];
    }
  const size_t o = pbase + static_cast<size_t>(oy) * a.W + ox;
  T* out = static_cast<T*>(a.out);
  const T* aux = static_cast<const T*>(a.aux);
  const T g = static_cast<T>(a.gain);
  const T tg = tanh(g);
  const T c1 = g / tg;
  switch (MODE) {
    case S_B:
    case S_BT: out[o] = s0; break;
    case S_B_MINUS: out[o] = s0 - aux[o]; break;
    case S_TANH_A: out[o] = tanh(g * s0) / tg; break;
    case S_TANH_WRES: {
      const T t = tanh(g * s0);
      out[o] = c1 * (T(1) - t * t) * (t / tg - aux[o]);
      break;
    }
    case S_TANH_JTW: {
      const T t = tanh(g * s0);
      out[o] = c1 * (T(1) - t * t) * aux[o];
      break;
    }
    case S_TANH_HESS: {
      const T t = tanh(g * s0);
      const T sech2 = T(1) - t * t;
      const T curv = T(-2) * g * g / tg * t * sech2;
      out[o] = s1 * (c1 * c1 * sech2 * sech2 + (t / tg - aux[o]) * curv);
      break;
    }
  }
}

// Output transform of a stencil mode for one pixel (s0 = k (*) in0, s1 = k (*) in1).
template <typename T, int MODE>
__device__ inline T stencil_out(T s0, T s1, T aux, T g, T tg) {
  const T c1 = g / tg;
  switch (MODE) {
    case S_B:
    case S_BT: return s0;
    case S_B_MINUS: return s0 - aux;
    case S_TANH_A: return tanh(g * s0) / tg;
    case S_TANH_WRES: {
      const T t = tanh(g * s0);
      return c1 * (T(1) - t * t) * (t / tg - aux);
    }
    case S_TANH_JTW: {
      const T t = tanh(g * s0);
      return c1 * (T(1) - t * t) * aux;
    }
    default: {  // S_TANH_HESS
      const T t = tanh(g * s0);
      const T sech2 = T(1) - t * t;
      const T curv = T(-2) * g * g / tg * t * sech2;
      return s1 * (c1 * c1 * sech2 * sech2 + (t / tg - aux) * curv);
    }
  }
}

// Square K x K taps (K odd, compile time): 16 x 64 output tiles, four
// horizontally adjacent outputs per thread sharing their K + 3 row reads, all
// tap loops unrolled (the taps then sit in scalar registers).
constexpr int kSNO = 4;                  // outputs per thread
constexpr int kSTY = 16, kSTX = 16 * kSNO;
template <typename T, int MODE, int K>
__global__ __launch_bounds__(kBlock) void stencil_k_kernel(StencilArgs a, Taps<T> taps) {
  constexpr int R = (K - 1) / 2, LH = kSTY + K - 1, LW = kSTX + K - 1;
  constexpr bool TWO = MODE == S_TANH_HESS;
  __shared__ T tile0[LH * LW];
  __shared__ T tile1[TWO ? LH * LW : 1];
  const int plane = blockIdx.z;
  if (a.gate && ((1 << a.gate[plane / a.plane_div]) & a.gate_mask) == 0) return;
  const int ty0 = blockIdx.y * kSTY, tx0 = blockIdx.x * kSTX;
  const size_t pbase = static_cast<size_t>(plane) * a.H * a.W;
  const T* in0 = static_cast<const T*>(a.in0) + pbase;
  const T* in1 = static_cast<const T*>(a.in1) + (TWO ? pbase : 0);
  for (int i = threadIdx.x; i < LH * LW; i += kBlock) {
    const int ly = i / LW, lx = i - (i / LW) * LW;
    const int gy = wrap1(ty0 - R + ly, a.H), gx = wrap1(tx0 - R + lx, a.W);
    const size_t src = static_cast<size_t>(gy) * a.W + gx;
    tile0[i] = in0[src];
    if (TWO) tile1[i] = in1[src];
  }
  __syncthreads();
  const int ly = threadIdx.x / (kSTX / kSNO), lx = (threadIdx.x % (kSTX / kSNO)) * kSNO;
  const int oy = ty0 + ly, ox = tx0 + lx;
  if (oy >= a.H || ox >= a.W) return;
  T s0[kSNO], s1[kSNO];
#pragma unroll
  for (int u = 0; u < kSNO; ++u) s0[u] = s1[u] = T(0);
#pragma unroll
  for (int p = 0; p < K; ++p) {
    T r0[K + kSNO - 1], r1[TWO ? K + kSNO - 1 : 1];
#pragma unroll
    for (int q = 0; q < K + kSNO - 1; ++q) {
      r0[q] = tile0[(ly + p) * LW + lx + q];
      if (TWO) r1[q] = tile1[(ly + p) * LW + lx + q];
    }
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const T kv = taps.k[p * K + q];
#pragma unroll
      for (int u = 0; u < kSNO; ++u) {
        s0[u] += kv * r0[q + u];
        if (TWO) s1[u] += kv * r1[q + u];
      }
    }
  }
  const T g = static_cast<T>(a.gain), tg = tanh(g);
  const T* aux = static_cast<const T*>(a.aux);
  T* out = static_cast<T*>(a.out);
  const size_t o = pbase + static_cast<size_t>(oy) * a.W + ox;
  const bool uses_aux = MODE == S_B_MINUS || MODE == S_TANH_WRES || MODE == S_TANH_JTW ||
                        MODE == S_TANH_HESS;
#pragma unroll
  for (int u = 0; u < kSNO; ++u)
    if (ox + u < a.W)
      out[o + u] = stencil_out<T, MODE>(s0[u], s1[u], uses_aux ? aux[o + u] : T(0), g, tg);
}

template <typename T, int K>
int stencil_k_launch(const StencilArgs& a, const Taps<T>& tp, hipStream_t s) {
  dim3 grid((a.W + kSTX - 1) / kSTX, (a.H + kSTY - 1) / kSTY, a.NP);
  switch (a.mode) {
    case S_B: stencil_k_kernel<T, S_B, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_BT: stencil_k_kernel<T, S_BT, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_B_MINUS: stencil_k_kernel<T, S_B_MINUS, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_A: stencil_k_kernel<T, S_TANH_A, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_WRES: stencil_k_kernel<T, S_TANH_WRES, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_JTW: stencil_k_kernel<T, S_TANH_JTW, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_HESS: stencil_k_kernel<T, S_TANH_HESS, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    default: return fail(IDQ_E_INVAL, "bad stencil mode");
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

// Rank-1 taps k[p][q] = u[p] v[q] (the Gaussian and box blurs): a horizontal
// pass over the staged tile into LDS, then a vertical one, 2K FMAs per output
// (plus the halo rows of the first pass) instead of K^2.
template <typename T>
struct SepTaps {
  T u[kMaxTap], v[kMaxTap];
};

template <typename T, int MODE, int K>
__global__ __launch_bounds__(kBlock) void stencil_sep_kernel(StencilArgs a, SepTaps<T> tp) {
  constexpr int R = (K - 1) / 2, LH = kSTY + K - 1, LW = kSTX + K - 1;
  constexpr bool TWO = MODE == S_TANH_HESS;
  __shared__ T tile0[LH * LW];
  __shared__ T tile1[TWO ? LH * LW : 1];
  __shared__ T hb0[LH * kSTX];
  __shared__ T hb1[TWO ? LH * kSTX : 1];
  const int plane = blockIdx.z;
  if (a.gate && ((1 << a.gate[plane / a.plane_div]) & a.gate_mask) == 0) return;
  const int ty0 = blockIdx.y * kSTY, tx0 = blockIdx.x * kSTX;
  const size_t pbase = static_cast<size_t>(plane) * a.H * a.W;
  const T* in0 = static_cast<const T*>(a.in0) + pbase;
  const T* in1 = static_cast<const T*>(a.in1) + (TWO ? pbase : 0);
  for (int i = threadIdx.x; i < LH * LW; i += kBlock) {
    const int ly = i / LW, lx = i - (i / LW) * LW;
    const int gy = wrap1(ty0 - R + ly, a.H), gx = wrap1(tx0 - R + lx, a.W);
    const size_t src = static_cast<size_t>(gy) * a.W + gx;
    tile0[i] = in0[src];
    if (TWO) tile1[i] = in1[src];
  }
  __syncthreads();
  // horizontal: hb[row][x] = sum_q v[q] tile[row][x + q], kSNO outputs per thread
  for (int i = threadIdx.x; i < LH * (kSTX / kSNO); i += kBlock) {
    const int ly = i / (kSTX / kSNO), lx = (i % (kSTX / kSNO)) * kSNO;
    T r0[K + kSNO - 1], r1[TWO ? K + kSNO - 1 : 1];
#pragma unroll
    for (int q = 0; q < K + kSNO - 1; ++q) {
      r0[q] = tile0[ly * LW + lx + q];
      if (TWO) r1[q] = tile1[ly * LW + lx + q];
    }
#pragma unroll
    for (int u = 0; u < kSNO; ++u) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int q = 0; q < K; ++q) {
        s0 += tp.v[q] * r0[q + u];
        if (TWO) s1 += tp.v[q] * r1[q + u];
      }
      hb0[ly * kSTX + lx + u] = s0;
      if (TWO) hb1[ly * kSTX + lx + u] = s1;
    }
  }
  __syncthreads();
  // vertical: out[y][x] = sum_p u[p] hb[y + p][x]
  const int ly = threadIdx.x / (kSTX / kSNO), lx = (threadIdx.x % (kSTX / kSNO)) * kSNO;
  const int oy = ty0 + ly, ox = tx0 + lx;
  if (oy >= a.H || ox >= a.W) return;
  T s0[kSNO], s1[kSNO];
#pragma unroll
  for (int u = 0; u < kSNO; ++u) s0[u] = s1[u] = T(0);
#pragma unroll
  for (int p = 0; p < K; ++p)
#pragma unroll
    for (int u = 0; u < kSNO; ++u) {
      s0[u] += tp.u[p] * hb0[(ly + p) * kSTX + lx + u];
      if (TWO) s1[u] += tp.u[p] * hb1[(ly + p) * kSTX + lx + u];
    }
  const T g = static_cast<T>(a.gain), tg = tanh(g);
  const T* aux = static_cast<const T*>(a.aux);
  T* out = static_cast<T*>(a.out);
  const size_t o = pbase + static_cast<size_t>(oy) * a.W + ox;
  const bool uses_aux = MODE == S_B_MINUS || MODE == S_TANH_WRES || MODE == S_TANH_JTW ||
                        MODE == S_TANH_HESS;
#pragma unroll
  for (int u = 0; u < kSNO; ++u)
    if (ox + u < a.W)
      out[o + u] = stencil_out<T, MODE>(s0[u], s1[u], uses_aux ? aux[o + u] : T(0), g, tg);
}

template <typename T, int K>
int stencil_sep_launch(const StencilArgs& a, const SepTaps<T>& tp, hipStream_t s) {
  dim3 grid((a.W + kSTX - 1) / kSTX, (a.H + kSTY - 1) / kSTY, a.NP);
  switch (a.mode) {
    case S_B: stencil_sep_kernel<T, S_B, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_BT: stencil_sep_kernel<T, S_BT, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_B_MINUS: stencil_sep_kernel<T, S_B_MINUS, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_A: stencil_sep_kernel<T, S_TANH_A, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_WRES: stencil_sep_kernel<T, S_TANH_WRES, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_JTW: stencil_sep_kernel<T, S_TANH_JTW, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_HESS: stencil_sep_kernel<T, S_TANH_HESS, K><<<grid, kBlock, 0, s>>>(a, tp); break;
    default: return fail(IDQ_E_INVAL, "bad stencil mode");
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

// k = u v^T within 1e-13 of the largest tap (u and v read from the row and
// column of that tap); rounding then differs from the direct sum by ~1 ulp
template <typename T>
bool separable(const double* k, int kh, int kw, bool flip, SepTaps<T>* tp) {
  int pr = 0, pc = 0;
  double m = 0.0;
  for (int p = 0; p < kh; ++p)
    for (int q = 0; q < kw; ++q)
      if (std::fabs(k[p * kw + q]) > m) {
        m = std::fabs(k[p * kw + q]);
        pr = p;
        pc = q;
      }
  if (!(m > 0.0)) return false;
  double u[kMaxTap], v[kMaxTap];
  for (int p = 0; p < kh; ++p) u[p] = k[p * kw + pc];
  for (int q = 0; q < kw; ++q) v[q] = k[pr * kw + q] / k[pr * kw + pc];
  for (int p = 0; p < kh; ++p)
    for (int q = 0; q < kw; ++q)
      if (std::fabs(k[p * kw + q] - u[p] * v[q]) > 1e-13 * m) return false;
  for (int p = 0; p < kh; ++p) tp->u[p] = static_cast<T>(u[flip ? kh - 1 - p : p]);
  for (int q = 0; q < kw; ++q) tp->v[q] = static_cast<T>(v[flip ? kw - 1 - q : q]);
  return true;
}

template <typename T>
int stencil_dispatch(const StencilArgs& a, const double* taps_host, hipStream_t s) {
  if (a.kh == a.kw && (a.kh == 9 || a.kh == 7)) {
    SepTaps<T> sp;
    if (separable(taps_host, a.kh, a.kw, a.mode == S_BT, &sp))
      return a.kh == 9 ? stencil_sep_launch<T, 9>(a, sp, s) : stencil_sep_launch<T, 7>(a, sp, s);
  }
  Taps<T> tp;
  const bool flip = a.mode == S_BT;
  for (int p = 0; p < a.kh; ++p)
    for (int q = 0; q < a.kw; ++q) {
      const int sp = flip ? a.kh - 1 - p : p, sq = flip ? a.kw - 1 - q : q;
      tp.k[p * a.kw + q] = static_cast<T>(taps_host[sp * a.kw + sq]);
    }
  if (a.kh == a.kw && a.kh == 9) return stencil_k_launch<T, 9>(a, tp, s);
  if (a.kh == a.kw && a.kh == 7) return stencil_k_launch<T, 7>(a, tp, s);
  if (a.kh == a.kw && a.kh == 5) return stencil_k_launch<T, 5>(a, tp, s);
  if (a.kh == a.kw && a.kh == 3) return stencil_k_launch<T, 3>(a, tp, s);
  dim3 grid((a.W + kTile - 1) / kTile, (a.H + kTile - 1) / kTile, a.NP);
  switch (a.mode) {
    case S_B: stencil_kernel<T, S_B><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_BT: stencil_kernel<T, S_BT><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_B_MINUS: stencil_kernel<T, S_B_MINUS><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_A: stencil_kernel<T, S_TANH_A><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_WRES: stencil_kernel<T, S_TANH_WRES><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_JTW: stencil_kernel<T, S_TANH_JTW><<<grid, kBlock, 0, s>>>(a, tp); break;
    case S_TANH_HESS: stencil_kernel<T, S_TANH_HESS><<<grid, kBlock, 0, s>>>(a, tp); break;
    default: return fail(IDQ_E_INVAL, "bad stencil mode");
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

// ---------------------------------------------------------------------------
// Elementwise kernels over n images of `per` elements (grid: blocks x images).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void extrap_kernel(const T* x, const T* xp, T* z,
                                                      const double* beta_eff, const int* gate,
                                                      int mask, long long per) {
  const int img = blockIdx.y;
  if (gate && ((1 << gate[img]) & mask) == 0) return;
  const T b = static_cast<T>(beta_eff[img]);
  const size_t base = static_cast<size_t>(img) * per;
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < per;
       i += (long long)gridDim.x * kBlock) {
    const T xv = x[base + i];
    z[base + i] = xv + b * (xv - xp[base + i]);
  }
}

// An image whose phase is not updated this step waits: its two iterate
// buffers trade places (the buffers' roles alternate with the step), so that
// the next step again finds x^k in its x operand and x^(k-1) in its xn one.
template <typename T>
__device__ inline void swap_wait(const UpdateArgs& a, size_t base, long long lo, long long hi) {
  T* x = const_cast<T*>(static_cast<const T*>(a.x)) + base;
  T* xn = static_cast<T*>(a.xn) + base;
  for (long long i = lo + threadIdx.x; i < hi; i += kBlock) {
    const T u = x[i], v = xn[i];
    x[i] = v;
    xn[i] = u;
  }
}

// update image `img` this step (else it is finished, or waits: swap_wait)
__device__ inline bool update_runs(const UpdateArgs& a, int img, bool* waits) {
  const int gv = a.gate ? a.gate[img] : G_LOW;
  *waits = a.gate && gv != G_DONE && ((1 << gv) & a.run_mask) == 0;
  return !a.gate || ((1 << gv) & a.run_mask) != 0;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void update_kernel(UpdateArgs a) {
  const int img = blockIdx.y;
  const int blk = blockIdx.x;
  const size_t base = static_cast<size_t>(img) * a.per;
  const long long chunk = (a.per + a.nblk - 1) / a.nblk;
  const long long lo = blk * chunk;
  const long long hi = lo + chunk < a.per ? lo + chunk : a.per;
  bool waits;
  if (!update_runs(a, img, &waits)) {
    if (waits) swap_wait<T>(a, base, lo, hi);
    return;
  }
  const T* x = static_cast<const T*>(a.x) + base;
  const T* z = static_cast<const T*>(a.z) + base;
  const T* gf = a.gf ? static_cast<const T*>(a.gf) + base : nullptr;
  const T* p = a.p ? static_cast<const T*>(a.p) + base : nullptr;
  const T* y = a.y ? static_cast<const T*>(a.y) + base : nullptr;
  const T* q = a.q ? static_cast<const T*>(a.q) + base : nullptr;
  T* xn = static_cast<T*>(a.xn) + base;
  const T tau = static_cast<T>(a.tau), lam = static_cast<T>(a.lambda);
  double s1 = 0.0, s0 = 0.0, nf = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += kBlock) {
    const T xv = x[i];
    T v = z[i];
    if (!a.given) {
      const T g = gf ? gf[i] : p[i] - y[i];
      const T qv = q ? q[i] : T(0);
      v -= tau * (g + lam * qv);
    }
    xn[i] = v;
    const double d = static_cast<double>(v) - static_cast<double>(xv);
    s1 += d * d;
    s0 += static_cast<double>(xv) * static_cast<double>(xv);
    if (!finite_v(v)) nf += 1.0;
  }
  block_sum3(s1, s0, nf);
  if (threadIdx.x == 0) {
    double* o = a.partials + (static_cast<size_t>(img) * a.nblk + blk) * 3;
    o[0] = s1;
    o[1] = s0;
    o[2] = nf;
  }
}

// float32 images of a multiple of 4 elements: 16-byte accesses, each thread
// issuing the loads of kU vectors before using any (the scalar loop above
// waits for every element's loads in turn)
constexpr int kU = 4;

__global__ __launch_bounds__(kBlock) void extrap_f4_kernel(const float4* x, const float4* xp,
                                                         float4* z, const double* beta_eff,
                                                         const int* gate, int mask,
                                                         long long per4) {
  const int img = blockIdx.y;
  if (gate && ((1 << gate[img]) & mask) == 0) return;
  const float b = static_cast<float>(beta_eff[img]);
  const size_t base = static_cast<size_t>(img) * per4;
  const long long step = static_cast<long long>(gridDim.x) * kBlock;
  for (long long i0 = blockIdx.x * static_cast<long long>(kBlock) + threadIdx.x; i0 < per4;
       i0 += step * kU) {
    float4 xv[kU], pv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * step;
      if (i < per4) {
        xv[u] = x[base + i];
        pv[u] = xp[base + i];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * step;
      if (i < per4)
        z[base + i] = make_float4(xv[u].x + b * (xv[u].x - pv[u].x), xv[u].y + b * (xv[u].y - pv[u].y),
                                  xv[u].z + b * (xv[u].z - pv[u].z), xv[u].w + b * (xv[u].w - pv[u].w));
    }
  }
}

__device__ inline void upd1(float x, float z, float g, float q, float tau, float lam, float& out,
                            double& s1, double& s0, double& nf) {
  const float v = z - tau * (g + lam * q);
  out = v;
  const double d = static_cast<double>(v) - static_cast<double>(x);
  s1 += d * d;
  s0 += static_cast<double>(x) * static_cast<double>(x);
  if (!isfinite(v)) nf += 1.0;
}

__global__ __launch_bounds__(kBlock) void update_f4_kernel(UpdateArgs a) {
  const int img = blockIdx.y;
  const int blk = blockIdx.x;
  const long long per4 = a.per / 4;
  const size_t base = static_cast<size_t>(img) * per4;
  const long long chunk = (per4 + a.nblk - 1) / a.nblk;
  const long long lo = blk * chunk;
  const long long hi = lo + chunk < per4 ? lo + chunk : per4;
  bool waits;
  if (!update_runs(a, img, &waits)) {
    if (waits) swap_wait<float4>(a, base, lo, hi);
    return;
  }
  const float4* x = static_cast<const float4*>(a.x) + base;
  const float4* z = static_cast<const float4*>(a.z) + base;
  const float4* gf = a.gf ? static_cast<const float4*>(a.gf) + base : nullptr;
  const float4* p = a.p ? static_cast<const float4*>(a.p) + base : nullptr;
  const float4* y = a.y ? static_cast<const float4*>(a.y) + base : nullptr;
  const float4* q = a.q ? static_cast<const float4*>(a.q) + base : nullptr;
  float4* xn = static_cast<float4*>(a.xn) + base;
  const float tau = static_cast<float>(a.tau), lam = static_cast<float>(a.lambda);
  double s1 = 0.0, s0 = 0.0, nf = 0.0;
  for (long long i0 = lo + threadIdx.x; i0 < hi; i0 += kBlock * kU) {
    float4 xv[kU], zv[kU], gv[kU], qv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * kBlock;
      if (i < hi) {
        xv[u] = x[i];
        zv[u] = z[i];
        if (a.given) {
          gv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else if (gf) {
          gv[u] = gf[i];
        } else {
          const float4 pv = p[i], yv = y[i];
          gv[u] = make_float4(pv.x - yv.x, pv.y - yv.y, pv.z - yv.z, pv.w - yv.w);
        }
        qv[u] = q ? q[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = i0 + u * kBlock;
      if (i < hi) {
        float4 o;
        upd1(xv[u].x, zv[u].x, gv[u].x, qv[u].x, tau, lam, o.x, s1, s0, nf);
        upd1(xv[u].y, zv[u].y, gv[u].y, qv[u].y, tau, lam, o.y, s1, s0, nf);
        upd1(xv[u].z, zv[u].z, gv[u].z, qv[u].z, tau, lam, o.z, s1, s0, nf);
        upd1(xv[u].w, zv[u].w, gv[u].w, qv[u].w, tau, lam, o.w, s1, s0, nf);
        xn[i] = o;
      }
    }
  }
  block_sum3(s1, s0, nf);
  if (threadIdx.x == 0) {
    double* o = a.partials + (static_cast<size_t>(img) * a.nblk + blk) * 3;
    o[0] = s1;
    o[1] = s0;
    o[2] = nf;
  }
}

// One wave per image: its lanes sum the update's block partials in a fixed
// order (strided, then a shuffle tree), lane 0 applies the rules.
__global__ __launch_bounds__(64) void finalize_kernel(FinalizeArgs a) {
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  ImgState s = a.st[i];
  if (s.done) return;
  if (((1 << s.prec) & a.run_mask) == 0) {
    // waiting: the update kernel moved x^k into the new buffer
    if (lane == 0) a.st[i].last_buf = a.buf_index;
    return;
  }
  double s1 = 0.0, s0 = 0.0, nf = 0.0;
  const double* p = a.partials + static_cast<size_t>(i) * a.nblk * 3;
  for (int b = lane; b < a.nblk; b += 64) {
    s1 += p[3 * b];
    s0 += p[3 * b + 1];
    nf += p[3 * b + 2];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off, 64);
    s0 += __shfl_down(s0, off, 64);
    nf += __shfl_down(nf, off, 64);
  }
  if (lane != 0) return;
  // averaging window of Alg. 1: K_0 = argmin_{floor(K/2) < k < K-1} ||x^{k+1} - x^k||,
  // the first such k on ties (strict <); k is this update's index (z^k -> x^{k+1})
  s.avg_snap = 0;
  if (a.avg_K > 0) {
    const int k = s.it;
    const double step = sqrt(s1);
    if (k > a.avg_K / 2 && k < a.avg_K - 1 && step < s.avg_best) {
      s.avg_best = step;
      s.avg_snap = k + 1;
    }
  }
  if (s.it == 0) s.norm0_sq = s0 > 0.0 ? s0 : s1;   // ||x^0||^2, or ||x^1||^2 from x^0 = 0
  s.it += 1;
  s.kr += 1;
  s.S += s1;
  const double rel = s0 > 0.0 ? sqrt(s1 / s0) : (s1 > 0.0 ? INFINITY : 0.0);
  s.rel = rel;
  s.last_buf = a.buf_index;
  int gate = s.prec;
  if (nf > 0.0 || !isfinite(s1)) {
    s.status = IDQ_ST_NONFINITE;
    s.done = 1;
  } else if (a.diverge_ratio > 0.0 && s.norm0_sq > 0.0 &&
             s0 > a.diverge_ratio * a.diverge_ratio * s.norm0_sq) {
    // the iterate norm grows geometrically when tau is too large for the
    // curvature (the relative step itself stays bounded)
    s.status = IDQ_ST_DIVERGED;
    s.done = 1;
  } else {
    s.beta_eff = a.beta;
    if (a.restart_B2 > 0.0 && static_cast<double>(s.kr) * s.S > a.restart_B2) {
      s.beta_eff = 0.0;
      s.kr = 0;
      s.S = 0.0;
      s.restarts += 1;
    }
    // precision phases: bf16 until rel < switch_tol or no new best for
    // switch_patience updates; then (optionally) split-bf16 until rel < tol or
    // the same stagnation rule; then the final arithmetic, which stops the image
    const bool low = s.prec == G_LOW, mid = s.prec == G_MID;
    if (low || mid) {
      if (low)
        s.it_low += 1;
      else
        s.it_mid += 1;
      if (rel < s.best_rel) {
        s.best_rel = rel;
        s.stall = 0;
      } else {
        s.stall += 1;
      }
      const bool next = low ? (rel < a.switch_tol || s.stall >= a.switch_patience)
                            : (rel < a.tol || s.stall >= a.switch_patience);
      if (next) {
        s.prec = (low && a.use_mid) ? G_MID : G_FINAL;
        s.best_rel = INFINITY;
        s.stall = 0;
      }
    }
    if (a.fixed_iters > 0) {
      if (s.it >= a.fixed_iters) {
        s.status = IDQ_ST_FIXED;
        s.done = 1;
      }
    } else if (!low && !mid && rel < a.tol) {
      s.status = IDQ_ST_CONVERGED;
      s.done = 1;
    } else if (s.it >= a.max_iter) {
      s.status = IDQ_ST_MAXITER;
      s.done = 1;
    }
    gate = s.prec;
  }
  // row = this image's own update count (steps it waited through have none)
  if (a.history && s.it - 1 < a.history_rows)
    a.history[static_cast<size_t>(s.it - 1) * a.n + i] = rel;
  a.st[i] = s;
  a.gate[i] = s.done ? G_DONE : gate;
  a.beta_eff[i] = s.beta_eff;
}

// zsum += z; xhat = zsum / avg_snap where the finalize marked a new best step.
// Only images this step updated (their count equals it_now) take part.
template <typename T>
__global__ __launch_bounds__(kBlock) void average_kernel(const T* z, double* zsum, T* xhat,
                                                       const ImgState* st, int it_now,
                                                       long long per) {
  const int img = blockIdx.y;
  if (st[img].it != it_now) return;
  const int snap = st[img].avg_snap;
  const size_t base = static_cast<size_t>(img) * per;
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < per;
       i += (long long)gridDim.x * kBlock) {
    const double acc = zsum[base + i] + static_cast<double>(z[base + i]);
    zsum[base + i] = acc;
    if (snap > 0) xhat[base + i] = static_cast<T>(acc / static_cast<double>(snap));
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void gather_kernel(const T* b0, const T* b1, T* out,
                                                      const ImgState* st, long long per,
                                                      int prev) {
  const int img = blockIdx.y;
  const size_t base = static_cast<size_t>(img) * per;
  int which = st[img].last_buf;
  if (prev && st[img].beta_eff != 0.0) which ^= 1;
  const T* src = which == 0 ? b0 : b1;
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < per;
       i += (long long)gridDim.x * kBlock)
    out[base + i] = src[base + i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void dot_stage1(const T* a, const T* b, long long count,
                                                   double* partials) {
  double s = 0.0, d1 = 0.0, d2 = 0.0;
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < count;
       i += (long long)gridDim.x * kBlock)
    s += static_cast<double>(a[i]) * static_cast<double>(b[i]);
  block_sum3(s, d1, d2);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void sum_stage2(const double* partials, int nblk,
                                                   double* out, int stride, double scale) {
  // one block per output: out[blockIdx.x] = scale * sum_j partials[blockIdx.x*stride + j]
  const double* p = partials + static_cast<size_t>(blockIdx.x) * stride;
  double s = 0.0, d1 = 0.0, d2 = 0.0;
  for (int j = threadIdx.x; j < nblk; j += kBlock) s += p[j];
  block_sum3(s, d1, d2);
  if (threadIdx.x == 0) out[blockIdx.x] = scale * s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void sqnorm_img_stage1(const T* a, long long per,
                                                          double* partials) {
  const int img = blockIdx.y;
  const size_t base = static_cast<size_t>(img) * per;
  double s = 0.0, d1 = 0.0, d2 = 0.0;
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < per;
       i += (long long)gridDim.x * kBlock) {
    const double v = static_cast<double>(a[base + i]);
    s += v * v;
  }
  block_sum3(s, d1, d2);
  if (threadIdx.x == 0) partials[static_cast<size_t>(img) * gridDim.x + blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scale_by_kernel(const T* a, T* out, long long count,
                                                        const double* scal, int mode) {
  const double sv = scal[0];
  const T f = static_cast<T>(mode == 0 ? sv : 1.0 / sqrt(sv));
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < count;
       i += (long long)gridDim.x * kBlock)
    out[i] = a[i] * f;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void axpbypcz_kernel(T al, const T* a, T be, const T* b,
                                                        T ga, const T* c, T* out,
                                                        long long count) {
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < count;
       i += (long long)gridDim.x * kBlock) {
    T v = al * a[i] + be * b[i];
    if (c) v += ga * c[i];
    out[i] = v;
  }
}

// ---------------------------------------------------------------------------
// Weight gradient partial sums: each thread owns one weight (or bias) slot and
// sums over one chunk of the flattened (image, pixel) range.
// ---------------------------------------------------------------------------
template <typename TM, typename TS, typename TA>
__device__ inline TM wg_load(const void* p, int fmt, int ni, int c, int C, int y, int x, int H,
                             int W) {
  if (fmt == F_NCHW)
    return ld<TM>(static_cast<const TS*>(p), ((static_cast<size_t>(ni) * C + c) * H + y) * W + x);
  return ld<TM>(static_cast<const TA*>(p), ((static_cast<size_t>(ni) * H + y) * W + x) * C + c);
}

template <typename TM, typename TS, typename TA>
__global__ __launch_bounds__(kBlock) void wgrad_kernel(WgradArgs a) {
  const int nw = a.CO * a.CI * 9;
  const int slot = blockIdx.x * kBlock + threadIdx.x;
  const int nslots = nw + (a.with_bias ? a.CO : 0);
  if (slot >= nslots) return;
  const long long total = static_cast<long long>(a.NI) * a.H * a.W;
  const long long chunk = (total + a.nchunk - 1) / a.nchunk;
  const long long lo = blockIdx.y * chunk;
  const long long hi = lo + chunk < total ? lo + chunk : total;
  double acc = 0.0;
  if (slot < nw) {
    const int co = slot / (a.CI * 9);
    const int ci = (slot / 9) % a.CI;
    const int t = slot % 9;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    for (long long q = lo; q < hi; ++q) {
      const int ni = static_cast<int>(q / (a.H * a.W));
      const int pix = static_cast<int>(q - static_cast<long long>(ni) * a.H * a.W);
      const int y = pix / a.W, x = pix - (pix / a.W) * a.W;
      const int yy = y + dy, xx = x + dx;
      if (yy < 0 || yy >= a.H || xx < 0 || xx >= a.W) continue;
      const TM g = wg_load<TM, TS, TA>(a.g, a.g_fmt, ni, co, a.CO, y, x, a.H, a.W);
      TM av = wg_load<TM, TS, TA>(a.a0, a.a_fmt, ni, ci, a.CI, yy, xx, a.H, a.W);
      if (a.a_pro == P_JVP) {
        const TM hd = wg_load<TM, TS, TA>(a.a1, a.a_fmt, ni, ci, a.CI, yy, xx, a.H, a.W);
        av = (a.act == IDQ_ACT_SOFTPLUS ? dsp_from_a(av) : TM(1)) * hd;
      }
      acc += static_cast<double>(g * av);
    }
  } else {
    const int co = slot - nw;
    for (long long q = lo; q < hi; ++q) {
      const int ni = static_cast<int>(q / (a.H * a.W));
      const int pix = static_cast<int>(q - static_cast<long long>(ni) * a.H * a.W);
      const int y = pix / a.W, x = pix - (pix / a.W) * a.W;
      acc += static_cast<double>(wg_load<TM, TS, TA>(a.g, a.g_fmt, ni, co, a.CO, y, x, a.H, a.W));
    }
  }
  a.partials[static_cast<size_t>(blockIdx.y) * nslots + slot] = acc;
}

// Sum of the chunk partials per slot: a block takes 64 slots; its 4 waves each
// add every 4th chunk in order, then wave 0 adds the 4 sums in a fixed order,
// so the result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(kBlock) void reduce_chunks_kernel(const double* partials, int nchunk,
                                                             int count, double scale, T* out,
                                                             int accumulate) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (i < count)
    for (int c = q; c < nchunk; c += 4) s += partials[static_cast<size_t>(c) * count + i];
  part[q][lane] = s;
  __syncthreads();
  if (q != 0 || i >= count) return;
  const double v = scale * ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]));
  out[i] = accumulate ? static_cast<T>(static_cast<double>(out[i]) + v) : static_cast<T>(v);
}

// 16-byte vector access needs every image to start 16-byte aligned
inline bool vec4_ok(long long per, std::initializer_list<const void*> ptrs) {
  if (per % 4 != 0) return false;
  for (const void* p : ptrs)
    if (p && (reinterpret_cast<uintptr_t>(p) & 15u) != 0) return false;
  return true;
}

inline int grid_for(long long per) {
  long long g = (per + kBlock - 1) / kBlock;
  if (g > 1024) g = 1024;
  return static_cast<int>(g < 1 ? 1 : g);
}

}  // namespace

int launch_stencil(const StencilArgs& a, const double* taps_host, int dtype, hipStream_t s) {
  if (a.kh > kMaxTap || a.kw > kMaxTap || a.kh % 2 == 0 || a.kw % 2 == 0)
    return fail(IDQ_E_INVAL, "blur taps must be odd and at most 9x9");
  if (a.NP > 65535) return fail(IDQ_E_INVAL, "too many planes");
  if (a.NP == 0) return IDQ_OK;
  return dtype == IDQ_F64 ? stencil_dispatch<double>(a, taps_host, s)
                          : stencil_dispatch<float>(a, taps_host, s);
}

int launch_extrap(const void* x, const void* xp, void* z, const double* beta_eff,
                  const int* gate, int mask, int n, long long per, int dtype, hipStream_t s) {
  if (dtype == IDQ_F32 && vec4_ok(per, {x, xp, z})) {
    const long long per4 = per / 4;
    long long g = (per4 + kBlock * kU - 1) / (kBlock * kU);
    dim3 grid(static_cast<int>(g < 1 ? 1 : (g > 256 ? 256 : g)), n);
    extrap_f4_kernel<<<grid, kBlock, 0, s>>>(static_cast<const float4*>(x),
                                             static_cast<const float4*>(xp),
                                             static_cast<float4*>(z), beta_eff, gate, mask, per4);
    IDQ_HIP(hipGetLastError());
    return IDQ_OK;
  }
  dim3 grid(grid_for(per), n);
  if (dtype == IDQ_F64)
    extrap_kernel<double><<<grid, kBlock, 0, s>>>(static_cast<const double*>(x),
                                                  static_cast<const double*>(xp),
                                                  static_cast<double*>(z), beta_eff, gate, mask, per);
  else
    extrap_kernel<float><<<grid, kBlock, 0, s>>>(static_cast<const float*>(x),
                                                 static_cast<const float*>(xp),
                                                 static_cast<float*>(z), beta_eff, gate, mask, per);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_update(const UpdateArgs& a, int dtype, hipStream_t s) {
  dim3 grid(a.nblk, a.n);
  if (dtype == IDQ_F64)
    update_kernel<double><<<grid, kBlock, 0, s>>>(a);
  else if (vec4_ok(a.per, {a.x, a.z, a.gf, a.p, a.y, a.q, a.xn}))
    update_f4_kernel<<<grid, kBlock, 0, s>>>(a);
  else
    update_kernel<float><<<grid, kBlock, 0, s>>>(a);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  finalize_kernel<<<a.n, 64, 0, s>>>(a);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_gather_result(const void* b0, const void* b1, void* out, const ImgState* st, int n,
                         long long per, int dtype, hipStream_t s, int prev) {
  dim3 grid(grid_for(per), n);
  if (dtype == IDQ_F64)
    gather_kernel<double><<<grid, kBlock, 0, s>>>(static_cast<const double*>(b0),
                                                  static_cast<const double*>(b1),
                                                  static_cast<double*>(out), st, per, prev);
  else
    gather_kernel<float><<<grid, kBlock, 0, s>>>(static_cast<const float*>(b0),
                                                 static_cast<const float*>(b1),
                                                 static_cast<float*>(out), st, per, prev);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_average(const void* z, double* zsum, void* xhat, const ImgState* st, int it_now,
                   int n, long long per, int dtype, hipStream_t s) {
  dim3 grid(grid_for(per), n);
  if (dtype == IDQ_F64)
    average_kernel<double><<<grid, kBlock, 0, s>>>(static_cast<const double*>(z), zsum,
                                                   static_cast<double*>(xhat), st, it_now, per);
  else
    average_kernel<float><<<grid, kBlock, 0, s>>>(static_cast<const float*>(z), zsum,
                                                  static_cast<float*>(xhat), st, it_now, per);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_dot(const void* a, const void* b, long long count, int dtype, double* partials,
               int nblk, double* out, hipStream_t s) {
  if (dtype == IDQ_F64)
    dot_stage1<double><<<nblk, kBlock, 0, s>>>(static_cast<const double*>(a),
                                               static_cast<const double*>(b), count, partials);
  else
    dot_stage1<float><<<nblk, kBlock, 0, s>>>(static_cast<const float*>(a),
                                              static_cast<const float*>(b), count, partials);
  sum_stage2<<<1, kBlock, 0, s>>>(partials, nblk, out, nblk, 1.0);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_half_sqnorm_per_image(const void* a, int n, long long per, int dtype,
                                 double* partials, int nblk, double* out, hipStream_t s) {
  dim3 grid(nblk, n);
  if (dtype == IDQ_F64)
    sqnorm_img_stage1<double><<<grid, kBlock, 0, s>>>(static_cast<const double*>(a), per, partials);
  else
    sqnorm_img_stage1<float><<<grid, kBlock, 0, s>>>(static_cast<const float*>(a), per, partials);
  sum_stage2<<<n, kBlock, 0, s>>>(partials, nblk, out, nblk, 0.5);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_scale_by(const void* a, void* out, long long count, const double* scal, int mode,
                    int dtype, hipStream_t s) {
  const int g = grid_for(count);
  if (dtype == IDQ_F64)
    scale_by_kernel<double><<<g, kBlock, 0, s>>>(static_cast<const double*>(a),
                                                 static_cast<double*>(out), count, scal, mode);
  else
    scale_by_kernel<float><<<g, kBlock, 0, s>>>(static_cast<const float*>(a),
                                                static_cast<float*>(out), count, scal, mode);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_axpbypcz(double alpha, const void* a, double beta, const void* b, double gamma,
                    const void* c, void* out, long long count, int dtype, hipStream_t s) {
  const int g = grid_for(count);
  if (dtype == IDQ_F64)
    axpbypcz_kernel<double><<<g, kBlock, 0, s>>>(alpha, static_cast<const double*>(a), beta,
                                                 static_cast<const double*>(b), gamma,
                                                 static_cast<const double*>(c),
                                                 static_cast<double*>(out), count);
  else
    axpbypcz_kernel<float><<<g, kBlock, 0, s>>>(
        static_cast<float>(alpha), static_cast<const float*>(a), static_cast<float>(beta),
        static_cast<const float*>(b), static_cast<float>(gamma), static_cast<const float*>(c),
        static_cast<float*>(out), count);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_wgrad(const WgradArgs& a, int prec, hipStream_t s) {
  if (wgrad_mfma_supported(a, prec)) return launch_wgrad_mfma(a, prec, s);
  const int nslots = a.CO * a.CI * 9 + (a.with_bias ? a.CO : 0);
  dim3 grid((nslots + kBlock - 1) / kBlock, a.nchunk);
  if (prec == PREC_F64)
    wgrad_kernel<double, double, double><<<grid, kBlock, 0, s>>>(a);
  else if (prec == PREC_F32)
    wgrad_kernel<float, float, float><<<grid, kBlock, 0, s>>>(a);
  else
    wgrad_kernel<float, float, bf16><<<grid, kBlock, 0, s>>>(a);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_reduce_chunks(const double* partials, int nchunk, int count, double scale, void* out,
                         int accumulate, int dtype, hipStream_t s) {
  static_assert(kBlock == 256, "reduce_chunks_kernel takes 4 waves");
  if (count <= 0) return IDQ_OK;
  const int g = (count + 63) / 64;
  if (dtype == IDQ_F64)
    reduce_chunks_kernel<double><<<g, kBlock, 0, s>>>(partials, nchunk, count, scale,
                                                      static_cast<double*>(out), accumulate);
  else
    reduce_chunks_kernel<float><<<g, kBlock, 0, s>>>(partials, nchunk, count, scale,
                                                     static_cast<float*>(out), accumulate);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

}  // namespace idq
