// Learned warm start x0 = y + W_phi(y) for the fixed-point iteration (any x^0
// may start Alg. 1; this one is trained on the solver's own fixed points).
//
// 2-level conv encoder-decoder, 3x3 zero-padded convs, SoftPlus after every
// conv but the last:
//   e1 = sp(conv 3->32 (y)), e2 = sp(conv 32->32 (e1))        full resolution
//   p  = avgpool2x2(e2)                                         half resolution
//   e3..e6 = sp(conv 32->64), 3 x sp(conv 64->64)
//   c  = concat(nearest-upsample(e6) [64], e2 [32])             full resolution
//   d1 = sp(conv 96->32 (c)), d2 = sp(conv 32->32 (d1)), x0 = y + conv 32->3 (d2)
// Every conv runs on the library's implicit-GEMM kernels (bf16 or fp32 matrix
// cores).  Training: mean squared error against the target, backward through
// the same kernels (transposed convs, pooling / upsampling adjoints), weight
// gradients, Adam on float32 master weights, then the packed weight copies are
// rebuilt on the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

namespace {

constexpr int kWsLayers = 9;
constexpr int kWsCi[kWsLayers] = {3, 32, 32, 64, 64, 64, 96, 32, 32};
constexpr int kWsCo[kWsLayers] = {32, 32, 64, 64, 64, 64, 32, 32, 3};

struct WsLayer {
  int ci = 0, co = 0;
  size_t woff = 0, boff = 0;     // offsets in the packed parameter vector
  void* dfwd[3] = {};            // direct [co][ci][9] float (bf16-rounded for bf16)
  void* dtr[3] = {};             // direct transposed [ci][co][9]
  void* mfwd[3] = {};            // fragment-ordered (k_conv_mfma.h)
  void* mtr[3] = {};
};

}  // namespace

struct idq_ws {
  int device = 0;
  long long nparams = 0;
  float* master = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  int t = 0;
  int packed_version[3] = {-1, -1, -1};
  int version = 0;
  WsLayer L[kWsLayers];
  idq::Workspace ws;
};

namespace idq {

namespace {

constexpr int kB = 256;

enum WsSlot {
  S_E1, S_E2, S_P, S_E3, S_E4, S_E5, S_E6, S_C, S_D1, S_D2,  // activations
  S_GOUT, S_G0, S_G1, S_G2, S_GC, S_GP, S_PART, S_WG, S_X0
};

// ---- device helpers -----------------------------------------------------------
template <typename TA>
__device__ inline float ldf(const TA* p, size_t i) {
  return static_cast<float>(p[i]);
}
template <>
__device__ inline float ldf<bf16>(const bf16* p, size_t i) {
  return bf2f(p[i]);
}
template <typename TA>
__device__ inline void stf(TA* p, size_t i, float v) {
  p[i] = static_cast<TA>(v);
}
template <>
__device__ inline void stf<bf16>(bf16* p, size_t i, float v) {
  p[i] = f2bf(v);
}

// Fragment-order weights of one conv pass from the float32 master copy
// (the device twin of pack_mfma_weights).  W: [co][ci][9]; the transposed pass
// uses Wt[o][c][t] = W[c][o][8 - t].
__global__ void pack_mfma_kernel(const float* W, int ci, int co, int transposed, int bf,
                                 void* dst, long long total) {
  const long long idx = static_cast<long long>(blockIdx.x) * kB + threadIdx.x;
  if (idx >= total) return;
  const int V = bf ? 8 : 4, KC = 4 * V;
  const int cie = transposed ? co : ci, coe = transposed ? ci : co;
  const int nj = (coe + 15) / 16;
  const int e = static_cast<int>(idx % V);
  const int l = static_cast<int>((idx / V) % 64);
  const int j = static_cast<int>((idx / (V * 64)) % nj);
  const int ch = static_cast<int>(idx / (static_cast<long long>(V) * 64 * nj));
  const int o = 16 * j + (l % 16);
  const int k = ch * KC + (l / 16) * V + e;
  float v = 0.f;
  if (o < coe && k < 9 * cie) {
    const int c = k % cie, t = k / cie;
    v = transposed ? W[(static_cast<size_t>(c) * ci + o) * 9 + 8 - t]
                   : W[(static_cast<size_t>(o) * ci + c) * 9 + t];
  }
  if (bf)
    static_cast<bf16*>(dst)[idx] = f2bf(v);
  else
    static_cast<float*>(dst)[idx] = v;
}

__global__ void pack_direct_kernel(const float* W, int ci, int co, int transposed, int bf,
                                   float* dst) {
  const int idx = blockIdx.x * kB + threadIdx.x;
  const int n = ci * co * 9;
  if (idx >= n) return;
  float v;
  if (!transposed) {
    v = W[idx];
  } else {  // dst [c][o][t] = W[o][c][8 - t]
    const int t = idx % 9, o = (idx / 9) % co, c = idx / (9 * co);
    v = W[(static_cast<size_t>(o) * ci + c) * 9 + 8 - t];
  }
  dst[idx] = bf ? round_bf(v) : v;
}

template <typename TA>
__global__ void pool_kernel(const TA* in, TA* out, int n, int h, int w, int C) {
  // in: [n][h][w][C], out: [n][h/2][w/2][C], average of each 2x2 block
  const long long total = static_cast<long long>(n) * (h / 2) * (w / 2) * C;
  for (long long i = static_cast<long long>(blockIdx.x) * kB + threadIdx.x; i < total;
       i += static_cast<long long>(gridDim.x) * kB) {
    const int c = static_cast<int>(i % C);
    long long q = i / C;
    const int x = static_cast<int>(q % (w / 2));
    q /= (w / 2);
    const int y = static_cast<int>(q % (h / 2));
    const int b = static_cast<int>(q / (h / 2));
    const size_t base = ((static_cast<size_t>(b) * h + 2 * y) * w + 2 * x) * C + c;
    const float s = ldf(in, base) + ldf(in, base + C) + ldf(in, base + static_cast<size_t>(w) * C) +
                    ldf(in, base + static_cast<size_t>(w) * C + C);
    stf(out, i, 0.25f * s);
  }
}

// c[b][y][x][0:64] = e6[b][y/2][x/2][0:64], c[b][y][x][64:96] = e2[b][y][x][0:32]:
// a copy in 16-byte vectors; blockIdx.x = image row (b, y), threads over
// (x, vector) of that row
template <typename TA>
__global__ void upcat_kernel(const TA* e6, const TA* e2, TA* c, int n, int h, int w) {
  constexpr int VPC = 16 / static_cast<int>(sizeof(TA));  // channels per vector
  constexpr int G = 96 / VPC;                            // vectors per pixel
  const int row = blockIdx.x;
  const int b = row / h, y = row - (row / h) * h;
  const int t = blockIdx.y * kB + threadIdx.x;
  if (t >= w * G) return;
  const int x = t / G, gi = t - (t / G) * G;
  const int ch0 = gi * VPC;
  const size_t pix = static_cast<size_t>(row) * w + x;
  const TA* src = ch0 < 64
      ? e6 + ((static_cast<size_t>(b) * (h / 2) + y / 2) * (w / 2) + x / 2) * 64 + ch0
      : e2 + pix * 32 + (ch0 - 64);
  *reinterpret_cast<uint4*>(c + pix * 96 + ch0) = *reinterpret_cast<const uint4*>(src);
}

// delta_e6 = sigma'(h) * (sum over the 2x2 block of gc[:, 0:64]), sigma' from a = e6
template <typename TA>
__global__ void upadj_delta_kernel(const TA* gc, const TA* e6, TA* out, int n, int h, int w,
                                   int fast) {
  const long long total = static_cast<long long>(n) * (h / 2) * (w / 2) * 64;
  for (long long i = static_cast<long long>(blockIdx.x) * kB + threadIdx.x; i < total;
       i += static_cast<long long>(gridDim.x) * kB) {
    const int ch = static_cast<int>(i % 64);
    long long q = i / 64;
    const int x = static_cast<int>(q % (w / 2));
    q /= (w / 2);
    const int y = static_cast<int>(q % (h / 2));
    const int b = static_cast<int>(q / (h / 2));
    float s = 0.f;
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx)
        s += ldf(gc, ((static_cast<size_t>(b) * h + 2 * y + dy) * w + 2 * x + dx) * 96 + ch);
    const float a = ldf(e6, i);
    stf(out, i, (fast ? dsp_from_a_fast(a) : dsp_from_a(a)) * s);
  }
}

// delta_e2 = sigma'(h) * (gc[:, 64:96] + 0.25 * gp[y/2][x/2]), sigma' from a = e2
template <typename TA>
__global__ void pooladj_delta_kernel(const TA* gc, const TA* gp, const TA* e2, TA* out, int n,
                                     int h, int w, int fast) {
  const long long total = static_cast<long long>(n) * h * w * 32;
  for (long long i = static_cast<long long>(blockIdx.x) * kB + threadIdx.x; i < total;
       i += static_cast<long long>(gridDim.x) * kB) {
    const int ch = static_cast<int>(i % 32);
    const long long pix = i / 32;
    const int x = static_cast<int>(pix % w);
    const int y = static_cast<int>((pix / w) % h);
    const int b = static_cast<int>(pix / (static_cast<long long>(w) * h));
    const float g = ldf(gc, static_cast<size_t>(pix) * 96 + 64 + ch) +
                    0.25f * ldf(gp, ((static_cast<size_t>(b) * (h / 2) + y / 2) * (w / 2) + x / 2) * 32 + ch);
    const float a = ldf(e2, i);
    stf(out, i, (fast ? dsp_from_a_fast(a) : dsp_from_a(a)) * g);
  }
}

// g = 2 (x0 - t) / count ; partial sums of (x0 - t)^2 in float64
__global__ void mse_grad_kernel(const float* x0, const float* t, float* g, long long count,
                                double* partials) {
  __shared__ double red[kB];
  double s = 0.0;
  const float sc = 2.f / static_cast<float>(count);
  for (long long i = static_cast<long long>(blockIdx.x) * kB + threadIdx.x; i < count;
       i += static_cast<long long>(gridDim.x) * kB) {
    const float d = x0[i] - t[i];
    g[i] = sc * d;
    s += static_cast<double>(d) * static_cast<double>(d);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void adam_kernel(float* p, float* m, float* v, const float* g, long long n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const long long i = static_cast<long long>(blockIdx.x) * kB + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline int grid_of(long long n) {
  long long g = (n + kB - 1) / kB;
  if (g > 4096) g = 4096;
  return static_cast<int>(g < 1 ? 1 : g);
}

size_t asize(int prec) { return prec == PREC_BF16 ? 2 : 4; }

int ws_check(const idq_ws* ws, int n, int c, int h, int w, int prec) {
  if (!ws) return fail(IDQ_E_INVAL, "null warm-start handle");
  if (c != 3) return fail(IDQ_E_INVAL, "the warm-start network takes 3-channel images");
  if (n <= 0 || h <= 1 || w <= 1 || (h % 2) || (w % 2))
    return fail(IDQ_E_INVAL, "warm start needs positive, even image sizes");
  if (prec != IDQ_BF16 && prec != IDQ_F32) return fail(IDQ_E_INVAL, "warm start runs in bf16 or fp32");
  return IDQ_OK;
}

// Rebuild the packed weight copies for `prec` from the float32 master weights.
int ws_pack(idq_ws* ws, int prec, hipStream_t s) {
  if (ws->packed_version[prec] == ws->version) return IDQ_OK;
  const int bf = prec == PREC_BF16;
  for (int l = 0; l < kWsLayers; ++l) {
    WsLayer& L = ws->L[l];
    const float* W = ws->master + L.woff;
    const int nw = L.ci * L.co * 9;
    if (!L.dfwd[prec]) {
      IDQ_HIP(hipMalloc(&L.dfwd[prec], nw * 4));
      IDQ_HIP(hipMalloc(&L.dtr[prec], nw * 4));
      IDQ_HIP(hipMalloc(&L.mfwd[prec], pack_mfma_weights(prec, L.ci, L.co, nullptr, nullptr)));
      IDQ_HIP(hipMalloc(&L.mtr[prec], pack_mfma_weights(prec, L.co, L.ci, nullptr, nullptr)));
    }
    pack_direct_kernel<<<(nw + kB - 1) / kB, kB, 0, s>>>(W, L.ci, L.co, 0, bf,
                                                         static_cast<float*>(L.dfwd[prec]));
    pack_direct_kernel<<<(nw + kB - 1) / kB, kB, 0, s>>>(W, L.ci, L.co, 1, bf,
                                                         static_cast<float*>(L.dtr[prec]));
    const long long nf = static_cast<long long>(pack_mfma_weights(prec, L.ci, L.co, nullptr, nullptr)) /
                         (bf ? 2 : 4);
    const long long nt = static_cast<long long>(pack_mfma_weights(prec, L.co, L.ci, nullptr, nullptr)) /
                         (bf ? 2 : 4);
    pack_mfma_kernel<<<static_cast<int>((nf + kB - 1) / kB), kB, 0, s>>>(W, L.ci, L.co, 0, bf,
                                                                         L.mfwd[prec], nf);
    pack_mfma_kernel<<<static_cast<int>((nt + kB - 1) / kB), kB, 0, s>>>(W, L.ci, L.co, 1, bf,
                                                                         L.mtr[prec], nt);
  }
  IDQ_HIP(hipGetLastError());
  ws->packed_version[prec] = ws->version;
  return IDQ_OK;
}

ConvArgs ws_conv(const idq_ws* ws, int l, bool transposed, int prec, int n, int h, int w) {
  ConvArgs a{};
  const WsLayer& L = ws->L[l];
  a.NI = n;
  a.H = h;
  a.W = w;
  a.CI = transposed ? L.co : L.ci;
  a.CO = transposed ? L.ci : L.co;
  a.act = IDQ_ACT_SOFTPLUS;
  a.pro = P_NONE;
  a.wgt = transposed ? L.dtr[prec] : L.dfwd[prec];
  a.wmfma = transposed ? L.mtr[prec] : L.mfwd[prec];
  a.bias = transposed ? nullptr : ws->master + L.boff;
  a.img_div = 1;
  a.in_fmt = a.CI <= 4 ? F_NCHW : F_NHWC;
  a.out_fmt = a.CO <= 4 ? F_NCHW : F_NHWC;
  return a;
}

struct Acts {
  void *e1, *e2, *p, *e3, *e4, *e5, *e6, *c, *d1, *d2;
};

int ws_acts(idq_ws* ws, int n, int h, int w, int prec, Acts* A) {
  const size_t full = static_cast<size_t>(n) * h * w * asize(prec);
  const size_t half = static_cast<size_t>(n) * (h / 2) * (w / 2) * asize(prec);
  IDQ_TRY(ws->ws.get(S_E1, full * 32, &A->e1));
  IDQ_TRY(ws->ws.get(S_E2, full * 32, &A->e2));
  IDQ_TRY(ws->ws.get(S_P, half * 32, &A->p));
  IDQ_TRY(ws->ws.get(S_E3, half * 64, &A->e3));
  IDQ_TRY(ws->ws.get(S_E4, half * 64, &A->e4));
  IDQ_TRY(ws->ws.get(S_E5, half * 64, &A->e5));
  IDQ_TRY(ws->ws.get(S_E6, half * 64, &A->e6));
  IDQ_TRY(ws->ws.get(S_C, full * 96, &A->c));
  IDQ_TRY(ws->ws.get(S_D1, full * 32, &A->d1));
  IDQ_TRY(ws->ws.get(S_D2, full * 32, &A->d2));
  return IDQ_OK;
}

template <typename TA>
int ws_aux_launch(int which, const void* a0, const void* a1, const void* a2, void* out, int n,
                  int h, int w, int fast, hipStream_t s) {
  switch (which) {
    case 0: {
      const long long tot = static_cast<long long>(n) * (h / 2) * (w / 2) * 32;
      pool_kernel<TA><<<grid_of(tot), kB, 0, s>>>(static_cast<const TA*>(a0), static_cast<TA*>(out),
                                                  n, h, w, 32);
      break;
    }
    case 1: {
      const long long per_row = static_cast<long long>(w) * (96 / (16 / sizeof(TA)));
      const long long rows = static_cast<long long>(n) * h;
      if (rows > 0x7fffffff || (per_row + kB - 1) / kB > 65535)
        return fail(IDQ_E_INVAL, "warm-start image too large");
      dim3 grid(static_cast<unsigned>(rows), static_cast<unsigned>((per_row + kB - 1) / kB));
      upcat_kernel<TA><<<grid, kB, 0, s>>>(static_cast<const TA*>(a0),
                                           static_cast<const TA*>(a1), static_cast<TA*>(out),
                                           n, h, w);
      break;
    }
    case 2: {
      const long long tot = static_cast<long long>(n) * (h / 2) * (w / 2) * 64;
      upadj_delta_kernel<TA><<<grid_of(tot), kB, 0, s>>>(static_cast<const TA*>(a0),
                                                         static_cast<const TA*>(a1),
                                                         static_cast<TA*>(out), n, h, w, fast);
      break;
    }
    default: {
      const long long tot = static_cast<long long>(n) * h * w * 32;
      pooladj_delta_kernel<TA><<<grid_of(tot), kB, 0, s>>>(
          static_cast<const TA*>(a0), static_cast<const TA*>(a1), static_cast<const TA*>(a2),
          static_cast<TA*>(out), n, h, w, fast);
      break;
    }
  }
  IDQ_HIP(hipGetLastError());
  return IDQ_OK;
}

int ws_aux(int which, const void* a0, const void* a1, const void* a2, void* out, int n, int h,
           int w, int prec, hipStream_t s) {
  if (prec == PREC_BF16) return ws_aux_launch<bf16>(which, a0, a1, a2, out, n, h, w, 1, s);
  return ws_aux_launch<float>(which, a0, a1, a2, out, n, h, w, 0, s);
}

int ws_forward_pass(idq_ws* ws, const void* y, void* x0, int n, int h, int w, int prec, Acts* A,
                    hipStream_t s) {
  IDQ_TRY(ws_pack(ws, prec, s));
  IDQ_TRY(ws_acts(ws, n, h, w, prec, A));
  const int h2 = h / 2, w2 = w / 2;
  auto fwd = [&](int l, const void* in, void* out, int hh, int ww, int epi, const void* e0) {
    ConvArgs a = ws_conv(ws, l, false, prec, n, hh, ww);
    a.in0 = in;
    a.out0 = out;
    a.epi = epi;
    a.e0 = e0;
    return launch_conv(a, prec, s);
  };
  IDQ_TRY(fwd(0, y, A->e1, h, w, E_ACT, nullptr));
  IDQ_TRY(fwd(1, A->e1, A->e2, h, w, E_ACT, nullptr));
  IDQ_TRY(ws_aux(0, A->e2, nullptr, nullptr, A->p, n, h, w, prec, s));
  IDQ_TRY(fwd(2, A->p, A->e3, h2, w2, E_ACT, nullptr));
  IDQ_TRY(fwd(3, A->e3, A->e4, h2, w2, E_ACT, nullptr));
  IDQ_TRY(fwd(4, A->e4, A->e5, h2, w2, E_ACT, nullptr));
  IDQ_TRY(fwd(5, A->e5, A->e6, h2, w2, E_ACT, nullptr));
  IDQ_TRY(ws_aux(1, A->e6, A->e2, nullptr, A->c, n, h, w, prec, s));
  IDQ_TRY(fwd(6, A->c, A->d1, h, w, E_ACT, nullptr));
  IDQ_TRY(fwd(7, A->d1, A->d2, h, w, E_ACT, nullptr));
  IDQ_TRY(fwd(8, A->d2, x0, h, w, E_ADD, y));
  return IDQ_OK;
}

// Gradient of the mean squared error into ws->grad (float32, packed like the
// parameters); returns the loss through *loss when non-null (synchronous).
int ws_grad_impl(idq_ws* ws, const void* y, const void* target, int n, int h, int w, int prec,
                 double* loss, hipStream_t s) {
  Acts A;
  const long long cnt = static_cast<long long>(n) * 3 * h * w;
  void *x0, *gout, *part;
  IDQ_TRY(ws->ws.get(S_X0, cnt * 4, &x0));
  IDQ_TRY(ws->ws.get(S_GOUT, cnt * 4, &gout));
  IDQ_TRY(ws->ws.get(S_PART, 1024 * 8, &part));
  IDQ_TRY(ws_forward_pass(ws, y, x0, n, h, w, prec, &A, s));
  const int nb = 1024;
  mse_grad_kernel<<<nb, kB, 0, s>>>(static_cast<const float*>(x0), static_cast<const float*>(target),
                                    static_cast<float*>(gout), cnt, static_cast<double*>(part));
  IDQ_HIP(hipGetLastError());
  const int h2 = h / 2, w2 = w / 2;
  const size_t full = static_cast<size_t>(n) * h * w * asize(prec);
  const size_t half = static_cast<size_t>(n) * h2 * w2 * asize(prec);
  void *g0, *g1, *gc, *gp;
  IDQ_TRY(ws->ws.get(S_G0, full * 32, &g0));
  IDQ_TRY(ws->ws.get(S_G1, full * 32, &g1));
  IDQ_TRY(ws->ws.get(S_GC, full * 96, &gc));
  IDQ_TRY(ws->ws.get(S_GP, half * 32, &gp));
  // weight gradients: G_l (output gradient of layer l) correlated with its input
  auto wgrad = [&](int l, const void* G, const void* in, int hh, int ww) -> int {
    const WsLayer& L = ws->L[l];
    const int nslots = L.co * L.ci * 9 + L.co;
    const long long pix = static_cast<long long>(n) * hh * ww;
    const int nchunk = static_cast<int>(std::max<long long>(1, std::min<long long>(256, pix / 1024)));
    void* wp;
    IDQ_TRY(ws->ws.get(S_WG, static_cast<size_t>(nchunk) * nslots * 8, &wp));
    WgradArgs wa{};
    wa.NI = n;
    wa.H = hh;
    wa.W = ww;
    wa.CI = L.ci;
    wa.CO = L.co;
    wa.g_fmt = L.co <= 4 ? F_NCHW : F_NHWC;
    wa.a_fmt = L.ci <= 4 ? F_NCHW : F_NHWC;
    wa.a_pro = P_NONE;
    wa.act = IDQ_ACT_SOFTPLUS;
    wa.g = G;
    wa.a0 = in;
    wa.partials = static_cast<double*>(wp);
    wa.nchunk = nchunk;
    wa.with_bias = 1;
    IDQ_TRY(launch_wgrad(wa, prec, s));
    return launch_reduce_chunks(static_cast<double*>(wp), nchunk, nslots, 1.0, ws->grad + L.woff,
                                0, IDQ_F32, s);
  };
  auto bwd = [&](int l, const void* in, void* out, int hh, int ww, int epi, const void* e0) {
    ConvArgs a = ws_conv(ws, l, true, prec, n, hh, ww);
    a.in0 = in;
    a.out0 = out;
    a.epi = epi;
    a.e0 = e0;
    return launch_conv(a, prec, s);
  };
  // layer 8 (output conv, no activation): G_8 = gout
  IDQ_TRY(bwd(8, gout, g0, h, w, E_DELTA, A.d2));          // G_7
  IDQ_TRY(wgrad(8, gout, A.d2, h, w));
  IDQ_TRY(bwd(7, g0, g1, h, w, E_DELTA, A.d1));            // G_6
  IDQ_TRY(wgrad(7, g0, A.d1, h, w));
  IDQ_TRY(bwd(6, g1, gc, h, w, E_RAW, nullptr));           // d loss / d c
  IDQ_TRY(wgrad(6, g1, A.c, h, w));
  IDQ_TRY(ws_aux(2, gc, A.e6, nullptr, g0, n, h, w, prec, s));  // G_5 (half res)
  IDQ_TRY(bwd(5, g0, g1, h2, w2, E_DELTA, A.e5));          // G_4
  IDQ_TRY(wgrad(5, g0, A.e5, h2, w2));
  IDQ_TRY(bwd(4, g1, g0, h2, w2, E_DELTA, A.e4));          // G_3
  IDQ_TRY(wgrad(4, g1, A.e4, h2, w2));
  IDQ_TRY(bwd(3, g0, g1, h2, w2, E_DELTA, A.e3));          // G_2
  IDQ_TRY(wgrad(3, g0, A.e3, h2, w2));
  IDQ_TRY(bwd(2, g1, gp, h2, w2, E_RAW, nullptr));         // d loss / d p
  IDQ_TRY(wgrad(2, g1, A.p, h2, w2));
  IDQ_TRY(ws_aux(3, gc, gp, A.e2, g0, n, h, w, prec, s));  // G_1
  IDQ_TRY(bwd(1, g0, g1, h, w, E_DELTA, A.e1));            // G_0
  IDQ_TRY(wgrad(1, g0, A.e1, h, w));
  IDQ_TRY(wgrad(0, g1, y, h, w));
  if (loss) {
    std::vector<double> hp(nb);
    IDQ_HIP(hipMemcpyAsync(hp.data(), part, nb * 8, hipMemcpyDeviceToHost, s));
    IDQ_HIP(hipStreamSynchronize(s));
    double tot = 0.0;
    for (double v : hp) tot += v;
    *loss = tot / static_cast<double>(cnt);
  }
  return IDQ_OK;
}

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(IDQ_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(IDQ_E_INVAL, "unexpected exception");
  }
}

long long ws_param_count() {
  long long n = 0;
  for (int l = 0; l < kWsLayers; ++l) n += static_cast<long long>(kWsCi[l]) * kWsCo[l] * 9 + kWsCo[l];
  return n;
}

}  // namespace

int ws_forward_internal(idq_ws* ws, const void* y, void* x0, int n, int c, int h, int w, int prec,
                        hipStream_t s) {
  IDQ_TRY(ws_check(ws, n, c, h, w, prec));
  Acts A;
  return ws_forward_pass(ws, y, x0, n, h, w, prec, &A, s);
}

}  // namespace idq

using namespace idq;

extern "C" {

long long idq_ws_num_params(void) { return ws_param_count(); }

int idq_ws_create(idq_ws** out, const double* params, long long count, int device) {
  return guarded([&]() -> int {
    if (!out || !params) return fail(IDQ_E_INVAL, "null argument");
    *out = nullptr;
    if (count != ws_param_count()) return fail(IDQ_E_INVAL, "warm-start parameter count mismatch");
    IDQ_HIP(hipSetDevice(device));
    auto* ws = new idq_ws();
    ws->device = device;
    ws->nparams = count;
    size_t off = 0;
    for (int l = 0; l < kWsLayers; ++l) {
      ws->L[l].ci = kWsCi[l];
      ws->L[l].co = kWsCo[l];
      ws->L[l].woff = off;
      off += static_cast<size_t>(kWsCi[l]) * kWsCo[l] * 9;
      ws->L[l].boff = off;
      off += kWsCo[l];
    }
    std::vector<float> f(count);
    for (long long i = 0; i < count; ++i) f[i] = static_cast<float>(params[i]);
    const size_t bytes = sizeof(float) * count;
    if (hipMalloc(&ws->master, bytes) != hipSuccess || hipMalloc(&ws->m, bytes) != hipSuccess ||
        hipMalloc(&ws->v, bytes) != hipSuccess || hipMalloc(&ws->grad, bytes) != hipSuccess) {
      idq_ws_destroy(ws);
      return fail(IDQ_E_NOMEM, "warm-start parameter allocation failed");
    }
    IDQ_HIP(hipMemcpy(ws->master, f.data(), bytes, hipMemcpyHostToDevice));
    IDQ_HIP(hipMemset(ws->m, 0, bytes));
    IDQ_HIP(hipMemset(ws->v, 0, bytes));
    *out = ws;
    return IDQ_OK;
  });
}

int idq_ws_destroy(idq_ws* ws) {
  if (!ws) return IDQ_OK;
  (void)hipSetDevice(ws->device);
  (void)hipDeviceSynchronize();
  for (auto& L : ws->L)
    for (int p = 0; p < 3; ++p)
      for (void* q : {L.dfwd[p], L.dtr[p], L.mfwd[p], L.mtr[p]})
        if (q) (void)hipFree(q);
  for (float* q : {ws->master, ws->m, ws->v, ws->grad})
    if (q) (void)hipFree(q);
  ws->ws.release();
  delete ws;
  return IDQ_OK;
}

int idq_ws_get_params(idq_ws* ws, double* params) {
  return guarded([&]() -> int {
    if (!ws || !params) return fail(IDQ_E_INVAL, "null argument");
    IDQ_HIP(hipSetDevice(ws->device));
    std::vector<float> f(ws->nparams);
    IDQ_HIP(hipDeviceSynchronize());
    IDQ_HIP(hipMemcpy(f.data(), ws->master, sizeof(float) * ws->nparams, hipMemcpyDeviceToHost));
    for (long long i = 0; i < ws->nparams; ++i) params[i] = f[i];
    return IDQ_OK;
  });
}

int idq_ws_set_params(idq_ws* ws, const double* params) {
  return guarded([&]() -> int {
    if (!ws || !params) return fail(IDQ_E_INVAL, "null argument");
    IDQ_HIP(hipSetDevice(ws->device));
    std::vector<float> f(ws->nparams);
    for (long long i = 0; i < ws->nparams; ++i) f[i] = static_cast<float>(params[i]);
    IDQ_HIP(hipDeviceSynchronize());
    IDQ_HIP(hipMemcpy(ws->master, f.data(), sizeof(float) * ws->nparams, hipMemcpyHostToDevice));
    ws->version += 1;
    return IDQ_OK;
  });
}

int idq_ws_forward(idq_ws* ws, const void* y, void* x0, int n, int c, int h, int w, int prec,
                   void* stream) {
  return guarded([&]() -> int {
    if (!y || !x0) return fail(IDQ_E_INVAL, "null argument");
    IDQ_TRY(ws_check(ws, n, c, h, w, prec));
    IDQ_HIP(hipSetDevice(ws->device));
    return ws_forward_internal(ws, y, x0, n, c, h, w, prec, static_cast<hipStream_t>(stream));
  });
}

int idq_ws_grad(idq_ws* ws, const void* y, const void* target, void* grad, int n, int c, int h,
                int w, int prec, double* loss, void* stream) {
  return guarded([&]() -> int {
    if (!y || !target || !grad) return fail(IDQ_E_INVAL, "null argument");
    IDQ_TRY(ws_check(ws, n, c, h, w, prec));
    IDQ_HIP(hipSetDevice(ws->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    IDQ_TRY(ws_grad_impl(ws, y, target, n, h, w, prec, loss, s));
    IDQ_HIP(hipMemcpyAsync(grad, ws->grad, sizeof(float) * ws->nparams, hipMemcpyDeviceToDevice, s));
    return IDQ_OK;
  });
}

int idq_ws_train_step(idq_ws* ws, const void* y, const void* target, int n, int c, int h, int w,
                      int prec, double lr, double* loss, void* stream) {
  return guarded([&]() -> int {
    if (!y || !target) return fail(IDQ_E_INVAL, "null argument");
    IDQ_TRY(ws_check(ws, n, c, h, w, prec));
    IDQ_HIP(hipSetDevice(ws->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    IDQ_TRY(ws_grad_impl(ws, y, target, n, h, w, prec, loss, s));
    ws->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, static_cast<float>(ws->t));
    const float c2 = 1.f - std::pow(b2, static_cast<float>(ws->t));
    adam_kernel<<<static_cast<int>((ws->nparams + kB - 1) / kB), kB, 0, s>>>(
        ws->master, ws->m, ws->v, ws->grad, ws->nparams, static_cast<float>(lr), b1, b2, 1e-8f, c1,
        c2);
    IDQ_HIP(hipGetLastError());
    ws->version += 1;
    return IDQ_OK;
  });
}

}  // extern "C"
