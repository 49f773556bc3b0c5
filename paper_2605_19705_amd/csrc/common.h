// Shared definitions of the i-DEQ HIP library (device helpers, error plumbing).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/idq.h"

namespace idq {

// ---------------------------------------------------------------------------
// bfloat16 storage: 16-bit payload, converted by round-to-nearest-even.
// ---------------------------------------------------------------------------
struct bf16 {
  uint16_t u;
};

__host__ __device__ inline float bf2f(bf16 v) {
  union { uint32_t i; float f; } c;
  c.i = static_cast<uint32_t>(v.u) << 16;
  return c.f;
}

__host__ __device__ inline bf16 f2bf(float f) {
  union { uint32_t i; float f; } c;
  c.f = f;
  uint32_t x = c.i;
  bf16 r;
  if ((x & 0x7f800000u) == 0x7f800000u && (x & 0x007fffffu)) {  // NaN stays NaN
    r.u = static_cast<uint16_t>((x >> 16) | 0x0040u);
    return r;
  }
  x += 0x7fffu + ((x >> 16) & 1u);
  r.u = static_cast<uint16_t>(x >> 16);
  return r;
}

__host__ __device__ inline float round_bf(float f) { return bf2f(f2bf(f)); }

// Load/store of an activation element of any storage type as math type TM.
template <typename TM, typename TS>
__device__ inline TM ld(const TS* p, size_t i) { return static_cast<TM>(p[i]); }
template <>
__device__ inline float ld<float, bf16>(const bf16* p, size_t i) { return bf2f(p[i]); }
template <typename TS, typename TM>
__device__ inline void st(TS* p, size_t i, TM v) { p[i] = static_cast<TS>(v); }
template <>
__device__ inline void st<bf16, float>(bf16* p, size_t i, float v) { p[i] = f2bf(v); }

// ---------------------------------------------------------------------------
// Activation (SoftPlus with beta = 1, no threshold) and its derivatives.
// ---------------------------------------------------------------------------
__device__ inline float softplus_f(float t) { return fmaxf(t, 0.f) + log1pf(expf(-fabsf(t))); }
__device__ inline double softplus_f(double t) { return fmax(t, 0.0) + log1p(exp(-fabs(t))); }
__device__ inline float sigmoid_f(float t) {
  float e = expf(-fabsf(t));
  return t >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
}
__device__ inline double sigmoid_f(double t) {
  double e = exp(-fabs(t));
  return t >= 0.0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}

// sigma'(h) and sigma''(h) recovered from a = softplus(h):
// sigma(h) = 1 - exp(-softplus(h)) = -expm1(-a).
__device__ inline float dsp_from_a(float a) { return -expm1f(-a); }
__device__ inline double dsp_from_a(double a) { return -expm1(-a); }
// Fast variants for bfloat16 passes (operands carry 8 significant bits): the
// bare hardware exp2 / log2 (v_exp_f32, v_log_f32) without range reduction.
__device__ inline float exp_fast(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ inline float log_fast(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }
__device__ inline float dsp_from_a_fast(float a) { return 1.f - exp_fast(-a); }
// float32 conv epilogues: the hardware exp2 / log2 (about 1 ulp each) without
// the library's range reduction; absolute error of a few 1e-8 on values of
// order one (for t << 0 softplus is e^t, below that error).
__device__ inline float softplus_hw(float t) {
  return fmaxf(t, 0.f) + log_fast(1.f + exp_fast(-fabsf(t)));
}
__device__ inline float dsp_from_a_hw(float a) { return 1.f - exp_fast(-a); }
// softplus(t) = max(t, 0) + log1p(u), u = exp(-|t|) in (0, 1], with log1p(u) =
// u P(u), P the degree-4 least-squares fit of log1p(u)/u on Chebyshev nodes of
// [0, 1] (relative error below 6e-5, far under the 2^-9 of bf16 storage): one
// transcendental instead of two.
__device__ inline float softplus_fast(float t) {
  const float u = exp_fast(-fabsf(t));
  float p = fmaf(0.04155111f, u, -0.15783838f);
  p = fmaf(p, u, 0.3065611f);
  p = fmaf(p, u, -0.49703084f);
  p = fmaf(p, u, 0.99994499f);
  return fmaf(p, u, fmaxf(t, 0.f));
}

// ---------------------------------------------------------------------------
// Errors: thread-local message, status codes of idq.h.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define IDQ_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::idq::fail(IDQ_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define IDQ_TRY(expr)            \
  do {                           \
    int s_ = (expr);             \
    if (s_ < 0) return s_;       \
  } while (0)

inline size_t elem_size(int dtype) { return dtype == IDQ_F64 ? 8 : (dtype == IDQ_F32 ? 4 : 2); }

}  // namespace idq
