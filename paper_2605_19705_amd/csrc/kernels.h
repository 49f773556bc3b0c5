// Kernel launch interfaces used by the host drivers (api.hip, ws.hip).
#pragma once

#include "common.h"

namespace idq {

// Arithmetic of a conv pass: storage and math types.
//   PREC_F64 : double everywhere
//   PREC_F32 : float everywhere
//   PREC_BF16: float state tensors, bfloat16 activations and operands,
//              float accumulation
//   PREC_SPLIT: float state tensors and activations; the 64-channel passes split
//              every operand into bf16 hi + lo parts and accumulate
//              hi*hi + lo*hi + hi*lo in float (the others run as PREC_F32)
enum Prec { PREC_F64 = IDQ_F64, PREC_F32 = IDQ_F32, PREC_BF16 = IDQ_BF16, PREC_SPLIT = IDQ_BF16X3 };
constexpr int kNumPrec = 4;

// Activation buffers of the network hold a_l = sigma(h_l) (not h_l): the
// SoftPlus is evaluated once, in the producing pass's epilogue, and the
// derivatives the backward passes need are recovered from a:
//   sigma'(h)  = 1 - exp(-softplus(h)) = -expm1(-a),   sigma''(h) = s (1 - s).
// Input transform applied while loading a conv operand.
enum Pro {
  P_NONE = 0,  // operand = in0
  P_JVP = 1,   // operand = sigma'(h) * in1, sigma' from in0 = a    (tangent a')
};

// Output transform of a conv pass (acc = sum over taps and input channels).
enum Epi {
  E_ACT = 0,    // out0 = sigma(acc + b)                   (a_l)
  E_RES = 1,    // out0 = e0 - (acc + b)                   (r = x - N(x))
  E_DELTA = 2,  // out0 = sigma'(h) * acc, from e0 = a     (backprop through sigma)
  E_SUB = 3,    // out0 = e0 - acc                         (grad g = r - J^T r)
  E_RAW = 4,    // out0 = acc
  E_DDOT = 5,   // out0 = sigma''(h) e1 e2 + sigma'(h) acc, out1 = sigma'(h) e2  (e0 = a)
  E_ADD = 6,    // out0 = e0 + (acc + b)                   (x0 = y + W(y))
};

enum Fmt { F_NCHW = 0, F_NHWC = 1 };

// One zero-padded 3x3 conv pass over NI images of H x W pixels.
// Weights `wgt` point at the layer's packed weights for the kernel family
// chosen by the launcher (see conv_weights_layout in api.hip).
struct ConvArgs {
  int NI, H, W, CI, CO;
  int in_fmt, out_fmt;
  int pro, epi, act;
  const void* in0;
  const void* in1;
  const void* wgt;      // direct: [co][ci][9] of the math type
  const void* wmfma;    // MFMA-packed weights (nullable)
  const void* bias;     // [co] of the math type (nullable => 0)
  void* out0;
  void* out1;
  const void* e0;
  const void* e1;
  const void* e2;
  const int* gate;      // per solver image phase gate (nullable => always run)
  int gate_mask;        // run image i iff (1 << gate[i]) & gate_mask
  int img_div;          // solver image = net image / img_div
  unsigned long long* work_px;  // nullable: += output pixels actually computed
  hipEvent_t ev0, ev1;  // nullable: timing events stamped by the launch itself
};

// Phase gate values written by the finalize kernel.
//   G_LOW: bf16 phase, G_MID: split-bf16 phase, G_FINAL: the solve's own
//   arithmetic (float32 after a bf16 start), which alone may stop an image.
enum Gate { G_DONE = 0, G_LOW = 1, G_FINAL = 2, G_MID = 3 };
constexpr int GM_ACTIVE = (1 << G_LOW) | (1 << G_FINAL) | (1 << G_MID);

__device__ inline bool gate_open(const int* gate, int mask, int img) {
  return gate == nullptr || ((1 << gate[img]) & mask) != 0;
}
// The same test for a workgroup-uniform image index, read through the scalar
// unit (the gate array is not written while a conv pass runs): a vector load
// here would make the wave wait for all of its outstanding stores as well.
__device__ inline bool gate_open_uniform(const int* gate, int mask, int img) {
  if (gate == nullptr) return true;
  typedef const __attribute__((address_space(4))) int* const_ptr;
  const const_ptr cg = (const_ptr)(gate);  // address-space cast: constant memory
  return ((1 << cg[img]) & mask) != 0;
}

int launch_conv(const ConvArgs& a, int prec, hipStream_t s);

// MFMA weight packing for a layer; returns bytes needed when dst == nullptr.
size_t pack_mfma_weights(int prec, int ci, int co, const double* w /*[co][ci][9]*/,
                         void* dst_host);
bool mfma_supported(int prec, int ci, int co);
// float32 vector-ALU kernel for image-facing outputs (k_conv_thin.hip)
bool thin_supported(const ConvArgs& a, int prec);
int launch_conv_thin(const ConvArgs& a, int prec, hipStream_t s);

// ---- stencils of the forward operator (circular, per plane) --------------
enum StencilMode {
  S_B = 0,          // out = B in0
  S_BT = 1,         // out = B^T in0
  S_B_MINUS = 2,    // out = B in0 - aux                          (A z - y)
  S_TANH_A = 3,     // out = tanh(g B in0) / tanh g
  S_TANH_WRES = 4,  // t = tanh(g B in0): out = c1 (1 - t^2) (t / tanh g - aux)
  S_TANH_JTW = 5,   // t = tanh(g B in0): out = c1 (1 - t^2) aux
  S_TANH_HESS = 6,  // t = tanh(g B in0), u = B in1:
                    //   out = u (c1^2 (1-t^2)^2 + (t/tanh g - aux) curv(t))
};

struct StencilArgs {
  int NP, H, W;             // planes (n * c), spatial
  int kh, kw;
  double gain;
  const void* in0;
  const void* in1;
  const void* aux;
  void* out;
  const int* gate;          // per solver image (nullable => always run)
  int gate_mask;            // run plane p iff (1 << gate[p / plane_div]) & gate_mask
  int plane_div;            // solver image = plane / plane_div
  int mode;
};
int launch_stencil(const StencilArgs& a, const double* taps_host, int dtype, hipStream_t s);

// ---- elementwise / reductions ---------------------------------------------
// z = x + beta_eff[img] * (x - xp) over n images of `per` elements (images
// with (1 << gate[img]) & mask only).
int launch_extrap(const void* x, const void* xp, void* z, const double* beta_eff,
                  const int* gate, int mask, int n, long long per, int dtype, hipStream_t s);

// Fused update of the i-DEQ step and per-block float64 partial sums:
//   xn = z - tau (gf + lambda q),  gf = (gf_is_point ? p - y : gf)
//   partials[img][blk] = { sum (xn - x)^2, sum x^2, nonfinite count }
struct UpdateArgs {
  int n;
  long long per;
  const void* x;
  const void* z;
  const void* gf;      // grad f, or nullptr when gf = p - y (identity A)
  const void* p;       // gradient point (identity A)
  const void* y;
  const void* q;       // grad g (nullable => 0)
  void* xn;
  double tau, lambda;
  const int* gate;
  int run_mask;        // update image i iff (1 << gate[i]) & run_mask
  double* partials;    // [n][nblk][3]
  int nblk;
  int given;           // 1: xn = z (the step was formed elsewhere, e.g. a proximal
                       //    step); gf, p, y, q, tau unused
};
int launch_update(const UpdateArgs& a, int dtype, hipStream_t s);

// Per-image bookkeeping after an update (restart, stop, precision phase).
struct ImgState {
  int it, kr, status, done;
  int prec, it_low, stall, restarts;
  int last_buf, it_mid, avg_snap, pad2;
  double S, rel, best_rel, beta_eff;
  double avg_best;      // averaging: smallest ||x^{k+1} - x^k|| over the window
  double norm0_sq;      // ||x^0||^2 (||x^1||^2 when x^0 = 0), for the blow-up test
};
struct FinalizeArgs {
  int n, nblk;
  const double* partials;
  ImgState* st;
  int* gate;
  double* beta_eff;
  double beta, tol, restart_B2, switch_tol;
  int max_iter, fixed_iters, switch_patience;
  int use_mid;          // the bf16 phase hands over to a split-bf16 phase first
  int run_mask;         // phases updated this step; other images wait unchanged
  int buf_index;        // ping-pong buffer holding the new iterate
  double* history;      // nullable: [update][n] relative residuals, `history_rows` rows
  int history_rows;
  int avg_K;            // > 0: averaging step over a run of avg_K updates (Alg. 1)
  double diverge_ratio; // > 0: ||x^k|| > diverge_ratio * ||x^0|| stops the image (DIVERGED)
};
int launch_finalize(const FinalizeArgs& a, hipStream_t s);
// Averaging step of Alg. 1, after each finalize of a run where every image
// updates on every step: zsum[img] += z[img] for the images this step updated
// (st.it == it_now); where the finalize marked a new smallest step in the
// window (st.avg_snap = k + 1 > 0), xhat[img] = zsum[img] / (k + 1).  zsum is
// float64 whatever the dtype.
int launch_average(const void* z, double* zsum, void* xhat, const ImgState* st, int it_now,
                   int n, long long per, int dtype, hipStream_t s);
// x_out[img] = bufs[st[img].last_buf][img]; with `prev` the iterate before it,
// bufs[1 - last_buf][img], or x_out itself where the last update restarted the
// inertia (beta_eff = 0), so that (x_out, prev) resumes the iteration exactly
int launch_gather_result(const void* b0, const void* b1, void* out, const ImgState* st,
                         int n, long long per, int dtype, hipStream_t s, int prev = 0);

// Batch float64 dot product <a, b> (deterministic two-stage); result in *out.
int launch_dot(const void* a, const void* b, long long count, int dtype, double* partials,
               int nblk, double* out, hipStream_t s);
// Per-image 0.5 * sum a^2 into out[img].
int launch_half_sqnorm_per_image(const void* a, int n, long long per, int dtype,
                                 double* partials, int nblk, double* out, hipStream_t s);
// out = a * scale[0] ^ {pow}  (pow = -1/2 => divide by sqrt)  ; generic axpby
int launch_scale_by(const void* a, void* out, long long count, const double* scal,
                    int mode, int dtype, hipStream_t s);
// out = alpha * a + beta * b + gamma * c (c nullable)
int launch_axpbypcz(double alpha, const void* a, double beta, const void* b, double gamma,
                    const void* c, void* out, long long count, int dtype, hipStream_t s);

// ---- pixelwise data terms (inpainting mask, Rician likelihood) -------------
enum DatafitMode {
  D_MASK_APPLY = 0,    // out = M . x
  D_MASK_GRAD = 1,     // out = M (x - y)
  D_MASK_PROX = 2,     // out = (u + tau M y) / (1 + tau M), u = x + a1 v (v nullable),
                       // M = 1 where the mask is null (identity operator)
  D_RICIAN_GRAD = 3,   // out = x / s^2 - (y / s^2) B(x y / s^2),  B = I_1 / I_0
  D_RICIAN_HESS = 4,   // out = (1 / s^2 - (y / s^2)^2 B'(x y / s^2)) v
  D_RICIAN_RATIO = 5,  // out = B(x)
};
struct DatafitArgs {
  int mode;
  long long count;     // elements of x / y / v / out
  long long plane;     // mask elements (h * w); the mask of element i is mask[i % plane]
  const void* x;
  const void* y;
  const void* v;
  const void* mask;    // h x w of the element type (mask modes)
  void* out;
  double inv_s2;       // 1 / sigma_y^2 (Rician modes)
  double tau;          // prox step
  double a1;           // D_MASK_PROX: weight of v in the prox operand
};
int launch_datafit(const DatafitArgs& a, int dtype, hipStream_t s);

// ---- 2-D DFT of image planes (k_fft.hip) ------------------------------------
constexpr int kFftMax = 1024;
enum FftDir { R_FWD = 0, R_INV = 1 };
enum FftColMode { C_FWD_MUL_INV = 0, C_FWD_MUL = 1, C_MUL_INV = 2 };
enum FftMult { M_MUL = 0, M_PROX = 1 };
struct FftArgs {
  int NP, H, W;                 // planes of H x W (powers of two, 4..kFftMax)
  int logh, logw;               // set by the launchers
  int rows_per_block, cols_per_block;  // set by the launchers
  // forward rows: real operand in0 + a1 in1 + a2 in2 (in1, in2 nullable)
  const void* in0;
  const void* in1;
  const void* in2;
  double a1, a2;
  void* cbuf;                   // complex NP x H x W work buffer (interleaved re, im)
  const void* cin;              // complex k-space operand of C_MUL_INV
  void* cout;                   // complex k-space output of C_FWD_MUL
  const void* mult;             // H x W real multiplier (nullable => 1)
  int mult_mode;                // M_MUL: scale * mult, M_PROX: scale / (1 + tau mult)
  double tau, scale;
  // inverse rows: out = scale_r * Re(row) + b0 * e0 (e0 nullable)
  void* out;
  const void* e0;
  double b0;
  double scale_r;
};
bool fft_supported(int h, int w);
int launch_fft_rows(FftArgs a, int dir, int dtype, hipStream_t s);
int launch_fft_cols(FftArgs a, int mode, int dtype, hipStream_t s);
struct BlurTaps {
  int kh, kw;
  double k[81];
};
// out[u * w + v] = |k^(u, v)|^2 of the centred taps on an h x w grid
int launch_blur_spectrum(void* out, int h, int w, const double* taps_host, int kh, int kw,
                         int dtype, hipStream_t s);

// ---- weight gradient:  dW[co][ci][tap] += scale * sum_p G[p][co] A[p+off][ci] ---
struct WgradArgs {
  int NI, H, W, CI, CO;
  int g_fmt, a_fmt;
  int a_pro, act;          // P_NONE | P_JVP on the A operand
  const void* g;           // gradient operand (c_out channels)
  const void* a0;          // A operand (c_in channels)
  const void* a1;          // tangent for P_JVP
  double* partials;        // [nchunk][CO*CI*9 + CO]
  int nchunk;
  int with_bias;           // also sum G over pixels into the bias slots
};
int launch_wgrad(const WgradArgs& a, int prec, hipStream_t s);
// float32 matrix-core form (k_wgrad_mfma.hip) for float32 or bf16 NHWC operands
// with CI, CO multiples of 16 and for the image-facing layers of the 32- and
// 64-channel nets; launch_wgrad takes it where supported.
bool wgrad_mfma_supported(const WgradArgs& a, int prec);
int launch_wgrad_mfma(const WgradArgs& a, int prec, hipStream_t s);
// out[i] (+)= scale * sum_chunk partials[chunk][i]; out of dtype, i < count
int launch_reduce_chunks(const double* partials, int nchunk, int count, double scale,
                         void* out, int accumulate, int dtype, hipStream_t s);

}  // namespace idq
