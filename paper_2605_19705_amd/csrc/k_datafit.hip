// Elementwise data terms of the forward models that act pixel by pixel:
//   * inpainting (App. D.3.2): A x = M . x with an h x w 0/1 pixel mask shared
//     by every channel; grad f = M (x - y), its Hessian M, and the closed-form
//     proximal step (v + tau M y) / (1 + tau M) (App. B, eq. red_prox);
//   * Rician denoising (App. D.3.3): f = x^2 / (2 s^2) - log I_0(x y / s^2),
//     grad f = x / s^2 - (y / s^2) B(x y / s^2) with B = I_1 / I_0, and the
//     diagonal Hessian 1 / s^2 - (y / s^2)^2 B'(t), B' = 1 - B / t - B^2.
// B is evaluated from the defining power series of I_0 and I_1 for
// |t| <= 30 and from their large-argument expansions above (Abramowitz &
// Stegun 9.6.10 and 9.7.1); the common factors cancel in the ratio, so
// neither is scaled.  Every kernel streams its operands once (HBM-bound).
#include "kernels.h"

namespace idq {

namespace {

constexpr int kBlk = 256;

template <typename T>
struct BesselCfg;
template <>
struct BesselCfg<float> {
  static constexpr int kSeriesMax = 64;   // (t/2)^2k / (k!)^2 below 2^-25 of the sum at t = 30
  static constexpr int kAsymTerms = 10;   // smallest term of the expansion at t = 30 ~ 1e-9
  static constexpr float kEps = 3e-8f;
};
template <>
struct BesselCfg<double> {
  static constexpr int kSeriesMax = 120;
  static constexpr int kAsymTerms = 28;   // terms fall as k / (2t) <= 28 / 60 at t = 30
  static constexpr double kEps = 1e-17;
};

// B(t) = I_1(t) / I_0(t), odd in t.
template <typename T>
__device__ inline T bessel_ratio(T t) {
  const T a = t < T(0) ? -t : t;
  T r;
  if (a <= T(30)) {
    const T q = T(0.25) * a * a;
    T s0 = T(1), s1 = T(1), t0 = T(1), t1 = T(1);
    for (int k = 1; k < BesselCfg<T>::kSeriesMax; ++k) {
      t0 *= q / T(k * k);
      t1 *= q / T(k * (k + 1));
      s0 += t0;
      s1 += t1;
      if (t0 < BesselCfg<T>::kEps * s0) break;
    }
    r = T(0.5) * a * s1 / s0;
  } else {
    const T inv8a = T(1) / (T(8) * a);
    T s0 = T(1), s1 = T(1), t0 = T(1), t1 = T(1);
#pragma unroll
    for (int k = 1; k < BesselCfg<T>::kAsymTerms; ++k) {
      const T odd2 = T((2 * k - 1) * (2 * k - 1));
      t0 *= -(T(0) - odd2) * inv8a / T(k);
      t1 *= -(T(4) - odd2) * inv8a / T(k);
      s0 += t0;
      s1 += t1;
    }
    r = s1 / s0;
  }
  return t < T(0) ? -r : r;
}

template <typename T>
__device__ inline T bessel_ratio_deriv(T t, T b) {
  return t == T(0) ? T(0.5) : T(1) - b / t - b * b;
}

template <typename T>
__global__ __launch_bounds__(kBlk) void datafit_kernel(DatafitArgs a) {
  const T* x = static_cast<const T*>(a.x);
  const T* y = static_cast<const T*>(a.y);
  const T* v = static_cast<const T*>(a.v);
  const T* m = static_cast<const T*>(a.mask);
  T* out = static_cast<T*>(a.out);
  const T s2i = static_cast<T>(a.inv_s2), tau = static_cast<T>(a.tau), a1 = static_cast<T>(a.a1);
  const long long total = a.count;
  for (long long i = blockIdx.x * static_cast<long long>(kBlk) + threadIdx.x; i < total;
       i += static_cast<long long>(gridDim.x) * kBlk) {
    const long long pix = i % a.plane;
    T o;
    switch (a.mode) {
      case D_MASK_APPLY:   // M . x
        o = m[pix] * x[i];
        break;
      case D_MASK_GRAD:    // M (x - y)
        o = m[pix] * (x[i] - y[i]);
        break;
      case D_MASK_PROX: {  // (u + tau M y) / (1 + tau M), u = x + a1 v
        const T u = v ? x[i] + a1 * v[i] : x[i];
        const T mv = m ? m[pix] : T(1);
        o = (u + tau * mv * y[i]) / (T(1) + tau * mv);
        break;
      }
      case D_RICIAN_GRAD: {  // x / s^2 - (y / s^2) B(x y / s^2)
        const T xv = x[i], yv = y[i];
        o = s2i * (xv - yv * bessel_ratio(xv * yv * s2i));
        break;
      }
      case D_RICIAN_HESS: {  // (1 / s^2 - (y / s^2)^2 B'(t)) v
        const T xv = x[i], yv = y[i], t = xv * yv * s2i;
        const T ys = yv * s2i;
        o = (s2i - ys * ys * bessel_ratio_deriv(t, bessel_ratio(t))) * v[i];
        break;
      }
      case D_RICIAN_RATIO:  // B(x) (exposed for its own parity test)
        o = bessel_ratio(x[i]);
        break;
      default:
        o = T(0);
    }
    out[i] = o;
  }
}

}  // namespace

int launch_datafit(const DatafitArgs& a, int dtype, hipStream_t s) {
  if (a.count <= 0) return IDQ_OK;
  if (a.plane <= 0) return fail(IDQ_E_INVAL, "datafit: bad plane size");
  long long g = (a.count + kBlk - 1) / kBlk;
  if (g > 4096) g = 4096;
  if (dtype == IDQ_F64)
    datafit_kernel<double><<<static_cast<int>(g), kBlk, 0, s>>>(a);
  else
    datafit_kernel<float><<<static_cast<int>(g), kBlk, 0, s>>>(a);
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

}  // namespace idq
