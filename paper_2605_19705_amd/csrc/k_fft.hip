// Two-dimensional discrete Fourier transforms of image planes for the
// operators that the DFT diagonalises:
//   * the MRI operator A x = M . F x (App. D.3.1) with F the unitary 2-D DFT:
//     grad f = F^H M_s F x - A^T y for real x, M_s(k) = (M(k) + M(-k)) / 2;
//   * the closed-form proximal steps (App. B, eq. red_prox) of the MRI term and
//     of the circular blur, (I + tau A^T A)^{-1} (v + tau A^T y), whose
//     multipliers in frequency are 1 / (1 + tau M_s) and 1 / (1 + tau |k^|^2).
//
// A plane of h x w (both powers of two, 4..1024) is transformed in two passes
// over HBM, rows and then columns, each a radix-2 decimation-in-time FFT held
// in LDS: operands are loaded once, coalesced, into bit-reversed LDS slots,
// log2(N) butterfly stages run between workgroup barriers, and the result is
// stored once.  The column pass does the forward transform, the multiplier and
// the inverse transform on the same LDS tile, so a gradient or a prox costs
// three passes: forward rows (real in, complex out), the fused column pass, and
// inverse rows (complex in, real part out, with the epilogue).  Twiddles are
// evaluated per workgroup in float64 (sincospi) and rounded to the element type.
#include <algorithm>

#include "kernels.h"

namespace idq {

namespace {

constexpr int kFftThreads = 256;

template <typename T>
struct C2 {
  T re, im;
};

template <typename T>
__device__ inline C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

__device__ inline int bitrev(int j, int logn) { return static_cast<int>(__brev(j) >> (32 - logn)); }

// tw[j] = exp(-2 pi i j / n), j < n / 2 (computed by threads of the block)
template <typename T>
__device__ inline void make_twiddles(C2<T>* tw, int n) {
  for (int j = threadIdx.x; j < n / 2; j += blockDim.x) {
    double sv, cv;
    sincospi(-2.0 * j / n, &sv, &cv);
    tw[j] = {static_cast<T>(cv), static_cast<T>(sv)};
  }
}

// In-place radix-2 DIT butterflies over `cnt` independent sequences of length
// n = 2^logn stored at buf + s * stride (bit-reversed order in, natural out).
// inverse: conjugate twiddles (no scaling).
template <typename T>
__device__ inline void fft_lds(C2<T>* buf, int stride, int cnt, int logn, const C2<T>* tw,
                               bool inverse) {
  const int n = 1 << logn;
  const int half = n >> 1;
  const int total = cnt * half;
  for (int s = 0; s < logn; ++s) {
    const int m = 1 << s;
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int seq = t / half;
      const int k = t - seq * half;
      const int pos = k & (m - 1);
      const int i0 = ((k >> s) << (s + 1)) + pos;
      const int i1 = i0 + m;
      C2<T> w = tw[pos << (logn - s - 1)];
      if (inverse) w.im = -w.im;
      C2<T>* b = buf + seq * stride;
      const C2<T> u = b[i0];
      const C2<T> v = cmul(b[i1], w);
      b[i0] = {u.re + v.re, u.im + v.im};
      b[i1] = {u.re - v.re, u.im - v.im};
    }
    __syncthreads();
  }
}

// ---- row pass --------------------------------------------------------------
// Forward (R_FWD): real operand v = in0 + a1 in1 + a2 in2 (in1, in2 nullable)
// -> complex rows in cbuf.  Inverse (R_INV): complex rows of cbuf -> real part
// times `scale_r`, plus b0 * e0 (nullable), into out.
template <typename T, int DIR>
__global__ __launch_bounds__(kFftThreads) void fft_rows_kernel(FftArgs a) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  const int n = a.W, logn = a.logw;
  C2<T>* rows = tw + n / 2;
  const int stride = n + 1;
  const int plane = blockIdx.y;
  const int r0 = blockIdx.x * a.rows_per_block;
  const int nr = min(a.rows_per_block, a.H - r0);
  if (nr <= 0) return;
  make_twiddles(tw, n);
  const size_t pbase = static_cast<size_t>(plane) * a.H * a.W;
  if (DIR == R_FWD) {
    const T* in0 = static_cast<const T*>(a.in0);
    const T* in1 = static_cast<const T*>(a.in1);
    const T* in2 = static_cast<const T*>(a.in2);
    const T a1 = static_cast<T>(a.a1), a2 = static_cast<T>(a.a2);
    for (int t = threadIdx.x; t < nr * n; t += blockDim.x) {
      const int r = t / n, c = t - r * n;
      const size_t gi = pbase + static_cast<size_t>(r0 + r) * n + c;
      T v = in0[gi];
      if (in1) v += a1 * in1[gi];
      if (in2) v += a2 * in2[gi];
      rows[r * stride + bitrev(c, logn)] = {v, T(0)};
    }
  } else {
    const C2<T>* cb = static_cast<const C2<T>*>(a.cbuf);
    for (int t = threadIdx.x; t < nr * n; t += blockDim.x) {
      const int r = t / n, c = t - r * n;
      rows[r * stride + bitrev(c, logn)] = cb[pbase + static_cast<size_t>(r0 + r) * n + c];
    }
  }
  __syncthreads();
  fft_lds(rows, stride, nr, logn, tw, DIR == R_INV);
  if (DIR == R_FWD) {
    C2<T>* cb = static_cast<C2<T>*>(a.cbuf);
    for (int t = threadIdx.x; t < nr * n; t += blockDim.x) {
      const int r = t / n, c = t - r * n;
      cb[pbase + static_cast<size_t>(r0 + r) * n + c] = rows[r * stride + c];
    }
  } else {
    T* out = static_cast<T*>(a.out);
    const T* e0 = static_cast<const T*>(a.e0);
    const T scale = static_cast<T>(a.scale_r), b0 = static_cast<T>(a.b0);
    for (int t = threadIdx.x; t < nr * n; t += blockDim.x) {
      const int r = t / n, c = t - r * n;
      const size_t gi = pbase + static_cast<size_t>(r0 + r) * n + c;
      T v = scale * rows[r * stride + c].re;
      if (e0) v += b0 * e0[gi];
      out[gi] = v;
    }
  }
}

// ---- column pass -------------------------------------------------------------
// A workgroup holds `cols` adjacent columns of one plane (h values each).
// C_FWD_MUL_INV: forward DFT, multiply, inverse DFT (in place in cbuf);
// C_FWD_MUL    : forward DFT, multiply, store to cout (k-space output);
// C_MUL_INV    : multiply the k-space operand cin, inverse DFT, store to cbuf.
// The multiplier of element (ky, kx) is scale * mult[ky * W + kx] (M_MUL),
// scale / (1 + tau * mult[...]) (M_PROX), or scale (mult == nullptr).
template <typename T, int MODE>
__global__ __launch_bounds__(kFftThreads) void fft_cols_kernel(FftArgs a) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  const int n = a.H, logn = a.logh, cols = a.cols_per_block;
  C2<T>* tile = tw + n / 2;
  const int stride = n + 1;
  const int plane = blockIdx.y;
  const int c0 = blockIdx.x * cols;
  make_twiddles(tw, n);
  const size_t pbase = static_cast<size_t>(plane) * a.H * a.W;
  const C2<T>* src = static_cast<const C2<T>*>(MODE == C_MUL_INV ? a.cin : a.cbuf);
  const T* mult = static_cast<const T*>(a.mult);
  const T scale = static_cast<T>(a.scale), tau = static_cast<T>(a.tau);
  auto factor = [&](int r, int c) -> T {
    if (!mult) return scale;
    const T m = mult[static_cast<size_t>(r) * a.W + c0 + c];
    return a.mult_mode == M_PROX ? scale / (T(1) + tau * m) : scale * m;
  };
  for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
    const int r = t / cols, c = t - r * cols;
    C2<T> v = src[pbase + static_cast<size_t>(r) * a.W + c0 + c];
    if (MODE == C_MUL_INV) {
      const T f = factor(r, c);
      v.re *= f;
      v.im *= f;
    }
    tile[c * stride + bitrev(r, logn)] = v;
  }
  __syncthreads();
  if (MODE != C_MUL_INV) {
    fft_lds(tile, stride, cols, logn, tw, false);
    // multiply in natural order, then bit-reverse again for the inverse
    if (MODE == C_FWD_MUL) {
      C2<T>* dst = static_cast<C2<T>*>(a.cout);
      for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
        const int r = t / cols, c = t - r * cols;
        C2<T> v = tile[c * stride + r];
        const T f = factor(r, c);
        dst[pbase + static_cast<size_t>(r) * a.W + c0 + c] = {v.re * f, v.im * f};
      }
      return;
    }
    // C_FWD_MUL_INV: gather the products into a second copy in bit-reversed order
    C2<T>* tile2 = tile + cols * stride;
    for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
      const int r = t / cols, c = t - r * cols;
      C2<T> v = tile[c * stride + r];
      const T f = factor(r, c);
      tile2[c * stride + bitrev(r, logn)] = {v.re * f, v.im * f};
    }
    __syncthreads();
    tile = tile2;
  }
  fft_lds(tile, stride, cols, logn, tw, true);
  C2<T>* dst = static_cast<C2<T>*>(a.cbuf);
  for (int t = threadIdx.x; t < n * cols; t += blockDim.x) {
    const int r = t / cols, c = t - r * cols;
    dst[pbase + static_cast<size_t>(r) * a.W + c0 + c] = tile[c * stride + r];
  }
}

// |k^|^2 of a circular correlation with kh x kw taps (centred) on an h x w grid:
// k^(u, v) = sum_{a,b} k[a,b] exp(-2 pi i (u (a - ry) / h + v (b - rx) / w)),
// accumulated in float64 (the spectrum is computed once per image size).
template <typename T>
__global__ __launch_bounds__(kFftThreads) void blur_spectrum_kernel(T* out, int h, int w,
                                                                  BlurTaps taps) {
  const int total = h * w;
  const int ry = (taps.kh - 1) / 2, rx = (taps.kw - 1) / 2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int u = i / w, v = i - u * w;
    double re = 0.0, im = 0.0;
    for (int p = 0; p < taps.kh; ++p)
      for (int q = 0; q < taps.kw; ++q) {
        // phase in turns, reduced mod 1 exactly in integers
        const long long num = static_cast<long long>(u) * (((p - ry) % h + h) % h) * w +
                              static_cast<long long>(v) * (((q - rx) % w + w) % w) * h;
        const long long hw = static_cast<long long>(h) * w;
        double sv, cv;
        sincospi(-2.0 * static_cast<double>(num % hw) / static_cast<double>(hw), &sv, &cv);
        re += taps.k[p * taps.kw + q] * cv;
        im += taps.k[p * taps.kw + q] * sv;
      }
    out[i] = static_cast<T>(re * re + im * im);
  }
}

int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}

}  // namespace

bool fft_supported(int h, int w) {
  const int lh = log2_exact(h), lw = log2_exact(w);
  return lh >= 2 && lw >= 2 && h <= kFftMax && w <= kFftMax;
}

int launch_fft_rows(FftArgs a, int dir, int dtype, hipStream_t s) {
  if (!fft_supported(a.H, a.W)) return fail(IDQ_E_UNSUPPORTED, "FFT sizes must be powers of two in [4, 1024]");
  if (a.NP <= 0) return IDQ_OK;
  if (a.NP > 65535) return fail(IDQ_E_INVAL, "too many planes");
  a.logw = log2_exact(a.W);
  a.logh = log2_exact(a.H);
  const size_t es = dtype == IDQ_F64 ? 16 : 8;
  // up to 2048 complex values of rows per workgroup (16 KB float32, 32 KB float64)
  a.rows_per_block = a.W >= 2048 ? 1 : std::min(a.H, 2048 / a.W);
  const size_t lds = es * (a.W / 2 + static_cast<size_t>(a.rows_per_block) * (a.W + 1));
  dim3 grid((a.H + a.rows_per_block - 1) / a.rows_per_block, a.NP);
  if (dtype == IDQ_F64) {
    if (dir == R_FWD) fft_rows_kernel<double, R_FWD><<<grid, kFftThreads, lds, s>>>(a);
    else fft_rows_kernel<double, R_INV><<<grid, kFftThreads, lds, s>>>(a);
  } else {
    if (dir == R_FWD) fft_rows_kernel<float, R_FWD><<<grid, kFftThreads, lds, s>>>(a);
    else fft_rows_kernel<float, R_INV><<<grid, kFftThreads, lds, s>>>(a);
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_fft_cols(FftArgs a, int mode, int dtype, hipStream_t s) {
  if (!fft_supported(a.H, a.W)) return fail(IDQ_E_UNSUPPORTED, "FFT sizes must be powers of two in [4, 1024]");
  if (a.NP <= 0) return IDQ_OK;
  if (a.NP > 65535) return fail(IDQ_E_INVAL, "too many planes");
  a.logw = log2_exact(a.W);
  a.logh = log2_exact(a.H);
  const size_t es = dtype == IDQ_F64 ? 16 : 8;
  // 128-byte row segments per load (16 float32 or 8 float64 complex values),
  // fewer columns where the tile would exceed 64 KB of LDS
  int cols = dtype == IDQ_F64 ? 8 : 16;
  cols = std::min(cols, a.W);
  const int copies = mode == C_FWD_MUL_INV ? 2 : 1;
  while (cols > 1 && es * (a.H / 2 + static_cast<size_t>(copies) * cols * (a.H + 1)) > 65536) cols /= 2;
  a.cols_per_block = cols;
  const size_t lds = es * (a.H / 2 + static_cast<size_t>(copies) * cols * (a.H + 1));
  dim3 grid(a.W / cols, a.NP);
  if (dtype == IDQ_F64) {
    switch (mode) {
      case C_FWD_MUL_INV: fft_cols_kernel<double, C_FWD_MUL_INV><<<grid, kFftThreads, lds, s>>>(a); break;
      case C_FWD_MUL: fft_cols_kernel<double, C_FWD_MUL><<<grid, kFftThreads, lds, s>>>(a); break;
      case C_MUL_INV: fft_cols_kernel<double, C_MUL_INV><<<grid, kFftThreads, lds, s>>>(a); break;
      default: return fail(IDQ_E_INVAL, "bad FFT column mode");
    }
  } else {
    switch (mode) {
      case C_FWD_MUL_INV: fft_cols_kernel<float, C_FWD_MUL_INV><<<grid, kFftThreads, lds, s>>>(a); break;
      case C_FWD_MUL: fft_cols_kernel<float, C_FWD_MUL><<<grid, kFftThreads, lds, s>>>(a); break;
      case C_MUL_INV: fft_cols_kernel<float, C_MUL_INV><<<grid, kFftThreads, lds, s>>>(a); break;
      default: return fail(IDQ_E_INVAL, "bad FFT column mode");
    }
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int launch_blur_spectrum(void* out, int h, int w, const double* taps_host, int kh, int kw,
                         int dtype, hipStream_t s) {
  if (kh > 9 || kw > 9 || kh * kw > 81) return fail(IDQ_E_INVAL, "blur taps must be at most 9x9");
  BlurTaps t{};
  t.kh = kh;
  t.kw = kw;
  for (int i = 0; i < kh * kw; ++i) t.k[i] = taps_host[i];
  const int total = h * w;
  const int grid = std::max(1, std::min(1024, (total + kFftThreads - 1) / kFftThreads));
  if (dtype == IDQ_F64)
    blur_spectrum_kernel<double><<<grid, kFftThreads, 0, s>>>(static_cast<double*>(out), h, w, t);
  else
    blur_spectrum_kernel<float><<<grid, kFftThreads, 0, s>>>(static_cast<float*>(out), h, w, t);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

}  // namespace idq
