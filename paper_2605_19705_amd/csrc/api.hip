// C ABI of the i-DEQ library: context management, operator and regularizer
// calls, the inertial fixed-point solver (Alg. 1), the power iteration for the
// step size and the implicit / JFB backward pass (App. D.1).
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

namespace idq {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int Workspace::get(int slot, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  if (cap[slot] < bytes) {
    if (ptr[slot]) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return fail(IDQ_E_HIP, std::string("sync: ") + hipGetErrorString(e));
      (void)hipFree(ptr[slot]);
      ptr[slot] = nullptr;
      cap[slot] = 0;
    }
    size_t want = (bytes + 255) / 256 * 256;
    if (hipMalloc(&ptr[slot], want) != hipSuccess) {
      ptr[slot] = nullptr;
      return fail(IDQ_E_NOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    cap[slot] = want;
  }
  *out = ptr[slot];
  return IDQ_OK;
}

void Workspace::release() {
  for (int i = 0; i < W_NSLOTS; ++i) {
    if (ptr[i]) (void)hipFree(ptr[i]);
    ptr[i] = nullptr;
    cap[i] = 0;
  }
}

int Profiler::take(int cls, ProfRec* r) {
  r->cls = cls;
  for (hipEvent_t* e : {&r->e0, &r->e1}) {
    if (!pool.empty()) {
      *e = pool.back();
      pool.pop_back();
    } else {
      // timing only: the elapsed times are read after the stream has been
      // synchronized, so the events need no system-scope fence (which would
      // write back and invalidate the caches around every timed launch)
      IDQ_HIP(hipEventCreateWithFlags(e, hipEventDisableSystemFence));
    }
  }
  return IDQ_OK;
}

int Profiler::begin(int cls, hipStream_t s, ProfRec* r) {
  IDQ_TRY(take(cls, r));
  IDQ_HIP(hipEventRecord(r->e0, s));
  return IDQ_OK;
}

int Profiler::end(ProfRec& r, hipStream_t s) {
  IDQ_HIP(hipEventRecord(r.e1, s));
  pending.push_back(r);
  return IDQ_OK;
}

int Profiler::flush() {
  for (ProfRec& r : pending) {
    IDQ_HIP(hipEventSynchronize(r.e1));
    float t = 0.f;
    IDQ_HIP(hipEventElapsedTime(&t, r.e0, r.e1));
    ms[r.cls] += t;
    launches[r.cls] += 1;
    pool.push_back(r.e0);
    pool.push_back(r.e1);
  }
  pending.clear();
  return IDQ_OK;
}

void Profiler::release() {
  flush();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
  if (dev_px) (void)hipFree(dev_px);
  dev_px = nullptr;
}

// Shape check shared by every entry point (declared in ctx.h).
int check_shape(const idq_ctx* ctx, int n, int c, int h, int w, Geometry* g) {
  if (n <= 0 || c <= 0 || h <= 0 || w <= 0) return fail(IDQ_E_INVAL, "non-positive shape");
  g->n = n;
  g->c = c;
  g->h = h;
  g->w = w;
  g->per = static_cast<long long>(c) * h * w;
  if (ctx->L > 0) {
    const int c0 = ctx->ch[0];
    if (c == c0) {
      g->NI = n;
      g->img_div = 1;
    } else if (c0 == 1) {
      g->NI = n * c;
      g->img_div = c;
    } else {
      return fail(IDQ_E_INVAL, "image channels " + std::to_string(c) + " do not match the network's " +
                                   std::to_string(c0));
    }
  } else {
    g->NI = n;
    g->img_div = 1;
  }
  if ((ctx->op_kind == IDQ_OP_INPAINT || ctx->op_kind == IDQ_OP_MRI) &&
      (h != ctx->mh || w != ctx->mw))
    return fail(IDQ_E_INVAL, "images are " + std::to_string(h) + " x " + std::to_string(w) +
                                 " but the operator's mask is " + std::to_string(ctx->mh) + " x " +
                                 std::to_string(ctx->mw));
  if (ctx->op_kind == IDQ_OP_MRI && !fft_supported(h, w))
    return fail(IDQ_E_UNSUPPORTED, "the MRI operator needs power-of-two h and w in [4, 1024]");
  return IDQ_OK;
}

// Stencil arguments of the forward operator for a geometry (declared in ctx.h).
StencilArgs stencil_base(const idq_ctx* ctx, const Geometry& g, const int* gate) {
  StencilArgs a{};
  a.NP = g.n * g.c;
  a.H = g.h;
  a.W = g.w;
  a.kh = ctx->kh;
  a.kw = ctx->kw;
  a.gain = ctx->gain;
  a.gate = gate;
  a.gate_mask = GM_ACTIVE;
  a.plane_div = g.c;
  return a;
}

namespace {

// Arithmetic a layer pass actually runs in: split-bf16 only where a split
// kernel exists, float32 (same float activations) elsewhere.
int eff_prec(int prec, int ci, int co) {
  return (prec == PREC_SPLIT && !mfma_supported(PREC_SPLIT, ci, co)) ? PREC_F32 : prec;
}

// Launch a conv pass, with device-time accounting when profiling is on.
int run_conv(idq_ctx* ctx, ConvArgs a, int prec, hipStream_t s) {
  prec = eff_prec(prec, a.CI, a.CO);
  if (!ctx->prof.on) return launch_conv(a, prec, s);
  int cls = PC_CONV_OTHER;
  if (a.CI == 64 && a.CO == 64 && prec != PREC_F64)
    cls = prec == PREC_BF16 ? PC_CONV_WIDE_BF16
                            : (prec == PREC_SPLIT ? PC_CONV_WIDE_SPLIT : PC_CONV_WIDE_F32);
  if (!ctx->prof.sample(cls)) return launch_conv(a, prec, s);
  a.work_px = ctx->prof.dev_px + cls;
  // the launcher stamps the events from the dispatch itself (hipExtLaunchKernel)
  // so that they time the kernel alone, not its launch latency
  ProfRec r;
  IDQ_TRY(ctx->prof.take(cls, &r));
  a.ev0 = r.e0;
  a.ev1 = r.e1;
  IDQ_TRY(launch_conv(a, prec, s));
  ctx->prof.pending.push_back(r);
  return IDQ_OK;
}

template <class F>
int profiled(idq_ctx* ctx, int cls, hipStream_t s, F&& f) {
  if (!ctx->prof.sample(cls)) return f();
  ProfRec r;
  IDQ_TRY(ctx->prof.begin(cls, s, &r));
  IDQ_TRY(f());
  return ctx->prof.end(r, s);
}

size_t math_size(int prec) { return prec == PREC_F64 ? 8 : 4; }
size_t act_size(int prec) { return prec == PREC_F64 ? 8 : (prec == PREC_BF16 ? 2 : 4); }

int upload(void** dst, const void* src, size_t bytes) {
  IDQ_HIP(hipMalloc(dst, bytes));
  IDQ_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return IDQ_OK;
}

void free_layers(idq_ctx* ctx) {
  for (auto& L : ctx->layers)
    for (int p = 0; p < kNumPrec; ++p) {
      void** all[] = {&L.fwd[p], &L.tr[p], &L.bias[p], &L.fwd_mfma[p], &L.tr_mfma[p]};
      for (void** q : all)
        if (*q) {
          (void)hipFree(*q);
          *q = nullptr;
        }
    }
}

// Pack every layer's weights for every arithmetic from ctx->params.
int pack_weights(idq_ctx* ctx) {
  free_layers(ctx);
  ctx->layers.assign(ctx->L, LayerW());
  size_t off = 0;
  for (int l = 0; l < ctx->L; ++l) {
    LayerW& lw = ctx->layers[l];
    const int ci = ctx->ch[l], co = ctx->ch[l + 1];
    lw.ci = ci;
    lw.co = co;
    const double* W = ctx->params.data() + off;
    const double* b = W + static_cast<size_t>(co) * ci * 9;
    off += static_cast<size_t>(co) * ci * 9 + co;
    // transposed-conv weights: Wt[c][o][t] = W[o][c][8 - t]
    std::vector<double> Wt(static_cast<size_t>(co) * ci * 9);
    for (int o = 0; o < co; ++o)
      for (int c = 0; c < ci; ++c)
        for (int t = 0; t < 9; ++t)
          Wt[(static_cast<size_t>(c) * co + o) * 9 + t] = W[(static_cast<size_t>(o) * ci + c) * 9 + 8 - t];
    const size_t nw = static_cast<size_t>(co) * ci * 9;
    IDQ_TRY(upload(&lw.fwd[PREC_F64], W, nw * 8));
    IDQ_TRY(upload(&lw.tr[PREC_F64], Wt.data(), nw * 8));
    IDQ_TRY(upload(&lw.bias[PREC_F64], b, co * 8));
    for (int prec : {PREC_F32, PREC_BF16}) {
      std::vector<float> f(nw), ft(nw), fb(co);
      for (size_t i = 0; i < nw; ++i) {
        f[i] = static_cast<float>(W[i]);
        ft[i] = static_cast<float>(Wt[i]);
        if (prec == PREC_BF16) {
          f[i] = round_bf(f[i]);
          ft[i] = round_bf(ft[i]);
        }
      }
      for (int o = 0; o < co; ++o) fb[o] = static_cast<float>(b[o]);
      IDQ_TRY(upload(&lw.fwd[prec], f.data(), nw * 4));
      IDQ_TRY(upload(&lw.tr[prec], ft.data(), nw * 4));
      IDQ_TRY(upload(&lw.bias[prec], fb.data(), co * 4));
      if (mfma_supported(prec, ci, co)) {
        std::vector<char> buf(pack_mfma_weights(prec, ci, co, W, nullptr));
        pack_mfma_weights(prec, ci, co, W, buf.data());
        IDQ_TRY(upload(&lw.fwd_mfma[prec], buf.data(), buf.size()));
      }
      if (mfma_supported(prec, co, ci)) {
        std::vector<char> buf(pack_mfma_weights(prec, co, ci, Wt.data(), nullptr));
        pack_mfma_weights(prec, co, ci, Wt.data(), buf.data());
        IDQ_TRY(upload(&lw.tr_mfma[prec], buf.data(), buf.size()));
      }
    }
    // split-bf16: hi/lo fragment copies where a split kernel exists, float bias
    {
      std::vector<float> fb(co);
      for (int o = 0; o < co; ++o) fb[o] = static_cast<float>(b[o]);
      IDQ_TRY(upload(&lw.bias[PREC_SPLIT], fb.data(), co * 4));
      if (mfma_supported(PREC_SPLIT, ci, co)) {
        std::vector<char> buf(pack_mfma_weights(PREC_SPLIT, ci, co, W, nullptr));
        pack_mfma_weights(PREC_SPLIT, ci, co, W, buf.data());
        IDQ_TRY(upload(&lw.fwd_mfma[PREC_SPLIT], buf.data(), buf.size()));
      }
      if (mfma_supported(PREC_SPLIT, co, ci)) {
        std::vector<char> buf(pack_mfma_weights(PREC_SPLIT, co, ci, Wt.data(), nullptr));
        pack_mfma_weights(PREC_SPLIT, co, ci, Wt.data(), buf.data());
        IDQ_TRY(upload(&lw.tr_mfma[PREC_SPLIT], buf.data(), buf.size()));
      }
    }
  }
  return IDQ_OK;
}

int check_prec(int dtype, int prec) {
  if (dtype != IDQ_F64 && dtype != IDQ_F32) return fail(IDQ_E_INVAL, "dtype must be IDQ_F64 or IDQ_F32");
  if (dtype == IDQ_F64 && prec != IDQ_F64)
    return fail(IDQ_E_INVAL, "float64 tensors need float64 conv arithmetic");
  if (dtype == IDQ_F32 && prec != IDQ_F32 && prec != IDQ_BF16 && prec != IDQ_BF16X3)
    return fail(IDQ_E_INVAL, "float32 tensors need F32, BF16 or BF16X3 conv arithmetic");
  return IDQ_OK;
}

size_t max_ch(const idq_ctx* ctx) {
  int m = 1;
  for (int l = 0; l <= ctx->L; ++l) m = std::max(m, ctx->ch[l]);
  return static_cast<size_t>(m);
}

ConvArgs conv_base(const idq_ctx* ctx, const Geometry& g, int l, bool transposed, int prec,
                   const int* gate, int mask) {
  ConvArgs a{};
  const LayerW& lw = ctx->layers[l];
  prec = transposed ? eff_prec(prec, lw.co, lw.ci) : eff_prec(prec, lw.ci, lw.co);
  a.NI = g.NI;
  a.H = g.h;
  a.W = g.w;
  a.CI = transposed ? lw.co : lw.ci;
  a.CO = transposed ? lw.ci : lw.co;
  a.act = ctx->act;
  a.wgt = transposed ? lw.tr[prec] : lw.fwd[prec];
  a.wmfma = transposed ? lw.tr_mfma[prec] : lw.fwd_mfma[prec];
  a.bias = transposed ? nullptr : lw.bias[prec];
  a.gate = gate;
  a.gate_mask = mask;
  a.img_div = g.img_div;
  return a;
}

// ---------------------------------------------------------------------------
// Regularizer passes
// ---------------------------------------------------------------------------

// Forward pass of N at p (state tensor): stores a_l = sigma(h_l) (l < L) and
// r = p - N(p).
int net_forward(idq_ctx* ctx, const Geometry& g, int prec, const void* p, void* r,
                const int* gate, int mask, hipStream_t s) {
  const int L = ctx->L;
  const size_t abytes = static_cast<size_t>(g.pix()) * max_ch(ctx) * act_size(prec);
  const void* prev = p;
  for (int l = 0; l < L; ++l) {
    ConvArgs a = conv_base(ctx, g, l, false, prec, gate, mask);
    a.in0 = prev;
    a.in_fmt = l == 0 ? F_NCHW : F_NHWC;
    a.pro = P_NONE;
    if (l == L - 1) {
      a.out_fmt = F_NCHW;
      a.epi = E_RES;
      a.e0 = p;
      a.out0 = r;
    } else {
      void* h;
      IDQ_TRY(ctx->ws.get(W_H0 + l, abytes, &h));
      a.out_fmt = F_NHWC;
      a.epi = E_ACT;
      a.out0 = h;
      prev = h;
    }
    IDQ_TRY(run_conv(ctx, a, prec, s));
  }
  return IDQ_OK;
}

// grad g(p) = r - J_N(p)^T r into q (state tensor); uses the buffers of net_forward.
int net_grad(idq_ctx* ctx, const Geometry& g, int prec, const void* p, void* q,
             const int* gate, int mask, hipStream_t s) {
  const int L = ctx->L;
  const size_t abytes = static_cast<size_t>(g.pix()) * max_ch(ctx) * act_size(prec);
  const size_t sbytes = static_cast<size_t>(g.n) * g.per * math_size(prec);
  void* r;
  IDQ_TRY(ctx->ws.get(W_R, sbytes, &r));
  IDQ_TRY(net_forward(ctx, g, prec, p, r, gate, mask, s));
  void *d0, *d1;
  IDQ_TRY(ctx->ws.get(W_TMP0, abytes, &d0));
  IDQ_TRY(ctx->ws.get(W_TMP1, abytes, &d1));
  const void* din = r;
  for (int l = L - 1; l >= 0; --l) {
    ConvArgs a = conv_base(ctx, g, l, true, prec, gate, mask);
    a.in0 = din;
    a.in_fmt = l == L - 1 ? F_NCHW : F_NHWC;
    a.pro = P_NONE;
    if (l == 0) {
      a.out_fmt = F_NCHW;
      a.epi = E_SUB;
      a.e0 = r;
      a.out0 = q;
    } else {
      void* h;
      IDQ_TRY(ctx->ws.get(W_H0 + l - 1, abytes, &h));
      void* o = (din == d0) ? d1 : d0;
      a.out_fmt = F_NHWC;
      a.epi = E_DELTA;
      a.e0 = h;
      a.out0 = o;
      din = o;
    }
    IDQ_TRY(run_conv(ctx, a, prec, s));
  }
  return IDQ_OK;
}

// Forward-over-reverse pass at x along w: Hw = H_g(x) w (state tensor).  Keeps
// h_l, h'_l, delta_l, delta'_l (l < L), r and r' in their workspace slots.
int net_hvp(idq_ctx* ctx, const Geometry& g, int prec, const void* x, const void* w, void* Hw,
            hipStream_t s) {
  const int L = ctx->L;
  const size_t abytes = static_cast<size_t>(g.pix()) * max_ch(ctx) * act_size(prec);
  const size_t sbytes = static_cast<size_t>(g.n) * g.per * math_size(prec);
  void *r, *rd, *t;
  IDQ_TRY(ctx->ws.get(W_R, sbytes, &r));
  IDQ_TRY(ctx->ws.get(W_RD, sbytes, &rd));
  IDQ_TRY(ctx->ws.get(W_T, abytes, &t));
  IDQ_TRY(net_forward(ctx, g, prec, x, r, nullptr, 0, s));
  // tangents
  const void* prev_h = nullptr;
  const void* prev_hd = w;
  for (int l = 0; l < L; ++l) {
    ConvArgs a = conv_base(ctx, g, l, false, prec, nullptr, 0);
    a.bias = nullptr;
    if (l == 0) {
      a.in0 = w;
      a.in_fmt = F_NCHW;
      a.pro = P_NONE;
    } else {
      a.in0 = prev_h;
      a.in1 = prev_hd;
      a.in_fmt = F_NHWC;
      a.pro = P_JVP;
    }
    if (l == L - 1) {
      a.out_fmt = F_NCHW;
      a.epi = E_SUB;
      a.e0 = w;
      a.out0 = rd;
    } else {
      void *h, *hd;
      IDQ_TRY(ctx->ws.get(W_H0 + l, abytes, &h));
      IDQ_TRY(ctx->ws.get(W_HD0 + l, abytes, &hd));
      a.out_fmt = F_NHWC;
      a.epi = E_RAW;
      a.out0 = hd;
      prev_h = h;
      prev_hd = hd;
    }
    IDQ_TRY(run_conv(ctx, a, prec, s));
  }
  // reverse pass for (delta, delta')
  const void* din = r;
  const void* ddin = rd;
  for (int l = L - 1; l >= 0; --l) {
    if (l == 0) {
      ConvArgs a = conv_base(ctx, g, 0, true, prec, nullptr, 0);
      a.in0 = ddin;
      a.in_fmt = L == 1 ? F_NCHW : F_NHWC;
      a.pro = P_NONE;
      a.out_fmt = F_NCHW;
      a.epi = E_SUB;
      a.e0 = rd;
      a.out0 = Hw;
      IDQ_TRY(run_conv(ctx, a, prec, s));
      break;
    }
    void *h, *hd, *dl, *ddl;
    IDQ_TRY(ctx->ws.get(W_H0 + l - 1, abytes, &h));
    IDQ_TRY(ctx->ws.get(W_HD0 + l - 1, abytes, &hd));
    IDQ_TRY(ctx->ws.get(W_DL0 + l - 1, abytes, &dl));
    IDQ_TRY(ctx->ws.get(W_DDL0 + l - 1, abytes, &ddl));
    ConvArgs a = conv_base(ctx, g, l, true, prec, nullptr, 0);
    a.in0 = din;
    a.in_fmt = l == L - 1 ? F_NCHW : F_NHWC;
    a.pro = P_NONE;
    a.out_fmt = F_NHWC;
    a.epi = E_RAW;
    a.out0 = t;
    IDQ_TRY(run_conv(ctx, a, prec, s));
    ConvArgs b = a;
    b.in0 = ddin;
    b.epi = E_DDOT;
    b.e0 = h;
    b.e1 = hd;
    b.e2 = t;
    b.out0 = ddl;
    b.out1 = dl;
    IDQ_TRY(run_conv(ctx, b, prec, s));
    din = dl;
    ddin = ddl;
  }
  return IDQ_OK;
}

// ---------------------------------------------------------------------------
// Forward operator passes
// ---------------------------------------------------------------------------
int copy_state(const void* src, void* dst, size_t bytes, hipStream_t s) {
  IDQ_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  return IDQ_OK;
}

int dt_index(int dtype) { return dtype == IDQ_F64 ? 0 : 1; }

bool has_prox(int kind) {
  return kind == IDQ_OP_IDENTITY || kind == IDQ_OP_BLUR_CIRC || kind == IDQ_OP_INPAINT ||
         kind == IDQ_OP_MRI;
}

// Elementwise data-term pass over the whole batch.
int datafit(idq_ctx* ctx, const Geometry& g, int dtype, int mode, const void* x, const void* y,
            const void* v, void* out, double tau, hipStream_t s) {
  DatafitArgs d{};
  d.mode = mode;
  d.count = static_cast<long long>(g.n) * g.per;
  d.plane = static_cast<long long>(g.h) * g.w;
  d.x = x;
  d.y = y;
  d.v = v;
  d.mask = ctx->mask_dev[dt_index(dtype)];
  d.out = out;
  d.inv_s2 = ctx->sigma > 0.0 ? 1.0 / (ctx->sigma * ctx->sigma) : 0.0;
  d.tau = tau;
  return launch_datafit(d, dtype, s);
}

FftArgs fft_base(const Geometry& g) {
  FftArgs f{};
  f.NP = g.n * g.c;
  f.H = g.h;
  f.W = g.w;
  f.scale = 1.0;
  f.scale_r = 1.0;
  return f;
}

// out = scale_r * Re(IDFT(mult . DFT(in0 + a1 in1 + a2 in2))) + b0 e0 over every
// plane, with unnormalised DFTs (mult_mode M_MUL: mult, M_PROX: 1 / (1 + tau mult)).
int fourier_pass(idq_ctx* ctx, const Geometry& g, int dtype, const void* in0, const void* in1,
                 double a1, const void* in2, double a2, const void* mult, int mult_mode,
                 double tau, double scale_r, const void* e0, double b0, void* out,
                 hipStream_t s) {
  void* cb;
  IDQ_TRY(ctx->ws.get(W_CPLX, static_cast<size_t>(g.n) * g.per * 2 * elem_size(dtype), &cb));
  FftArgs f = fft_base(g);
  f.in0 = in0;
  f.in1 = in1;
  f.a1 = a1;
  f.in2 = in2;
  f.a2 = a2;
  f.cbuf = cb;
  IDQ_TRY(launch_fft_rows(f, R_FWD, dtype, s));
  f.mult = mult;
  f.mult_mode = mult_mode;
  f.tau = tau;
  IDQ_TRY(launch_fft_cols(f, C_FWD_MUL_INV, dtype, s));
  f.out = out;
  f.e0 = e0;
  f.b0 = b0;
  f.scale_r = scale_r;
  return launch_fft_rows(f, R_INV, dtype, s);
}

// MRI: out = A^T v = Re(F^H (M v)) for complex k-space v (unitary DFT).
int mri_adjoint(idq_ctx* ctx, const Geometry& g, int dtype, const void* v, void* out,
                hipStream_t s) {
  void* cb;
  IDQ_TRY(ctx->ws.get(W_CPLX, static_cast<size_t>(g.n) * g.per * 2 * elem_size(dtype), &cb));
  FftArgs f = fft_base(g);
  f.cin = v;
  f.cbuf = cb;
  f.mult = ctx->mask_dev[dt_index(dtype)];
  f.mult_mode = M_MUL;
  IDQ_TRY(launch_fft_cols(f, C_MUL_INV, dtype, s));
  f.out = out;
  f.scale_r = 1.0 / std::sqrt(static_cast<double>(g.h) * g.w);
  return launch_fft_rows(f, R_INV, dtype, s);
}

// MRI: Ax = M . F x (complex, unitary DFT).
int mri_forward(idq_ctx* ctx, const Geometry& g, int dtype, const void* x, void* Ax,
                hipStream_t s) {
  void* cb;
  IDQ_TRY(ctx->ws.get(W_CPLX, static_cast<size_t>(g.n) * g.per * 2 * elem_size(dtype), &cb));
  FftArgs f = fft_base(g);
  f.in0 = x;
  f.cbuf = cb;
  IDQ_TRY(launch_fft_rows(f, R_FWD, dtype, s));
  f.cout = Ax;
  f.mult = ctx->mask_dev[dt_index(dtype)];
  f.mult_mode = M_MUL;
  f.scale = 1.0 / std::sqrt(static_cast<double>(g.h) * g.w);
  return launch_fft_cols(f, C_FWD_MUL, dtype, s);
}

// A^T y of a linear operator into the W_ATY slot (blur: B^T y; MRI: Re F^H M y).
int data_aty(idq_ctx* ctx, const Geometry& g, int dtype, const void* y, void** aty,
             hipStream_t s) {
  IDQ_TRY(ctx->ws.get(W_ATY, static_cast<size_t>(g.n) * g.per * elem_size(dtype), aty));
  if (ctx->op_kind == IDQ_OP_MRI) return mri_adjoint(ctx, g, dtype, y, *aty, s);
  if (ctx->op_kind == IDQ_OP_BLUR_CIRC) {
    StencilArgs b = stencil_base(ctx, g, nullptr);
    b.in0 = y;
    b.out = *aty;
    b.mode = S_BT;
    return launch_stencil(b, ctx->taps.data(), dtype, s);
  }
  return copy_state(y, *aty, static_cast<size_t>(g.n) * g.per * elem_size(dtype), s);
}

// |k^|^2 of the blur on the geometry's grid (computed once per size and dtype).
int blur_spectrum(idq_ctx* ctx, const Geometry& g, int dtype, const void** spec, hipStream_t s) {
  const int d = dt_index(dtype);
  if (ctx->spec_dev[d] == nullptr || ctx->spec_h[d] != g.h || ctx->spec_w[d] != g.w) {
    if (ctx->spec_dev[d]) {
      IDQ_HIP(hipStreamSynchronize(s));
      (void)hipFree(ctx->spec_dev[d]);
      ctx->spec_dev[d] = nullptr;
    }
    IDQ_HIP(hipMalloc(&ctx->spec_dev[d], static_cast<size_t>(g.h) * g.w * elem_size(dtype)));
    IDQ_TRY(launch_blur_spectrum(ctx->spec_dev[d], g.h, g.w, ctx->taps.data(), ctx->kh, ctx->kw,
                                 dtype, s));
    ctx->spec_h[d] = g.h;
    ctx->spec_w[d] = g.w;
  }
  *spec = ctx->spec_dev[d];
  return IDQ_OK;
}

// out = prox_{tau f(., y)}(v) with v = in0 + a1 in1 (in1 nullable), for the
// operators with a closed form (App. B, eq. red_prox; App. D.3.1-2).  For the
// Fourier forms `aty` = A^T y (from data_aty).
int prox_apply(idq_ctx* ctx, const Geometry& g, int dtype, const void* in0, const void* in1,
               double a1, const void* y, const void* aty, double tau, void* out,
               hipStream_t s) {
  switch (ctx->op_kind) {
    case IDQ_OP_IDENTITY:
    case IDQ_OP_INPAINT: {
      DatafitArgs d{};
      d.mode = D_MASK_PROX;
      d.count = static_cast<long long>(g.n) * g.per;
      d.plane = static_cast<long long>(g.h) * g.w;
      d.x = in0;
      d.v = in1;
      d.a1 = a1;
      d.y = y;
      d.mask = ctx->op_kind == IDQ_OP_INPAINT ? ctx->mask_dev[dt_index(dtype)] : nullptr;
      d.out = out;
      d.tau = tau;
      return launch_datafit(d, dtype, s);
    }
    case IDQ_OP_BLUR_CIRC: {
      const void* spec;
      IDQ_TRY(blur_spectrum(ctx, g, dtype, &spec, s));
      return fourier_pass(ctx, g, dtype, in0, in1, a1, aty, tau, spec, M_PROX, tau,
                          1.0 / (static_cast<double>(g.h) * g.w), nullptr, 0.0, out, s);
    }
    case IDQ_OP_MRI:
      return fourier_pass(ctx, g, dtype, in0, in1, a1, aty, tau, ctx->msym_dev[dt_index(dtype)],
                          M_PROX, tau, 1.0 / (static_cast<double>(g.h) * g.w), nullptr, 0.0,
                          out, s);
    default:
      return fail(IDQ_E_UNSUPPORTED, "this data term has no closed-form proximal step");
  }
}

// grad f(p, y) = J_A(p)^T (A(p) - y) into gf (not used for the identity,
// whose gradient p - y the update kernel forms itself unless `force`).  For
// MRI, `aty` = A^T y if already computed (else it is computed here).
int data_grad(idq_ctx* ctx, const Geometry& g, int dtype, const void* p, const void* y, void* gf,
              const int* gate, hipStream_t s, bool force, int mask = GM_ACTIVE,
              const void* aty = nullptr) {
  const size_t sbytes = static_cast<size_t>(g.n) * g.per * elem_size(dtype);
  switch (ctx->op_kind) {
    case IDQ_OP_IDENTITY:
      if (force) IDQ_TRY(launch_axpbypcz(1.0, p, -1.0, y, 0.0, nullptr, gf, g.n * g.per, dtype, s));
      return IDQ_OK;
    case IDQ_OP_INPAINT:
      return profiled(ctx, PC_STENCIL, s, [&] {
        return datafit(ctx, g, dtype, D_MASK_GRAD, p, y, nullptr, gf, 0.0, s);
      });
    case IDQ_OP_RICIAN:
      return profiled(ctx, PC_STENCIL, s, [&] {
        return datafit(ctx, g, dtype, D_RICIAN_GRAD, p, y, nullptr, gf, 0.0, s);
      });
    case IDQ_OP_MRI: {
      if (!aty) {
        void* t;
        IDQ_TRY(data_aty(ctx, g, dtype, y, &t, s));
        aty = t;
      }
      // F^H M_s F p - A^T y (the real part of F^H M (M F p - y) for real p)
      return profiled(ctx, PC_STENCIL, s, [&] {
        return fourier_pass(ctx, g, dtype, p, nullptr, 0.0, nullptr, 0.0,
                            ctx->msym_dev[dt_index(dtype)], M_MUL, 0.0,
                            1.0 / (static_cast<double>(g.h) * g.w), aty, -1.0, gf, s);
      });
    }
    default:
      break;
  }
  void* tmp;
  IDQ_TRY(ctx->ws.get(W_S, sbytes, &tmp));
  StencilArgs a = stencil_base(ctx, g, gate);
  a.gate_mask = mask;
  a.in0 = p;
  a.aux = y;
  a.out = tmp;
  a.mode = ctx->op_kind == IDQ_OP_BLUR_CIRC ? S_B_MINUS : S_TANH_WRES;
  IDQ_TRY(profiled(ctx, PC_STENCIL, s, [&] { return launch_stencil(a, ctx->taps.data(), dtype, s); }));
  StencilArgs b = stencil_base(ctx, g, gate);
  b.gate_mask = mask;
  b.in0 = tmp;
  b.out = gf;
  b.mode = S_BT;
  return profiled(ctx, PC_STENCIL, s, [&] { return launch_stencil(b, ctx->taps.data(), dtype, s); });
}

// Hessian of f at (x, y) along v into out.
int data_hvp(idq_ctx* ctx, const Geometry& g, int dtype, const void* x, const void* y,
             const void* v, void* out, hipStream_t s) {
  const size_t sbytes = static_cast<size_t>(g.n) * g.per * elem_size(dtype);
  switch (ctx->op_kind) {
    case IDQ_OP_IDENTITY:
      return copy_state(v, out, sbytes, s);
    case IDQ_OP_INPAINT:   // A^T A = M for a 0/1 mask
      return datafit(ctx, g, dtype, D_MASK_APPLY, v, nullptr, nullptr, out, 0.0, s);
    case IDQ_OP_RICIAN:
      return datafit(ctx, g, dtype, D_RICIAN_HESS, x, y, v, out, 0.0, s);
    case IDQ_OP_MRI:
      return fourier_pass(ctx, g, dtype, v, nullptr, 0.0, nullptr, 0.0,
                          ctx->msym_dev[dt_index(dtype)], M_MUL, 0.0,
                          1.0 / (static_cast<double>(g.h) * g.w), nullptr, 0.0, out, s);
    default:
      break;
  }
  void* tmp;
  IDQ_TRY(ctx->ws.get(W_S, sbytes, &tmp));
  StencilArgs a = stencil_base(ctx, g, nullptr);
  if (ctx->op_kind == IDQ_OP_BLUR_CIRC) {
    a.in0 = v;
    a.mode = S_B;
  } else {
    a.in0 = x;
    a.in1 = v;
    a.aux = y;
    a.mode = S_TANH_HESS;
  }
  a.out = tmp;
  IDQ_TRY(launch_stencil(a, ctx->taps.data(), dtype, s));
  StencilArgs b = stencil_base(ctx, g, nullptr);
  b.in0 = tmp;
  b.out = out;
  b.mode = S_BT;
  return launch_stencil(b, ctx->taps.data(), dtype, s);
}

// H_F(x) v = grad^2 f v + lambda H_g v into out.
int obj_hvp(idq_ctx* ctx, const Geometry& g, int dtype, int prec, const void* x, const void* y,
            const void* v, double lambda, void* out, hipStream_t s) {
  const size_t sbytes = static_cast<size_t>(g.n) * g.per * elem_size(dtype);
  void *hf, *hg;
  IDQ_TRY(ctx->ws.get(W_HF, sbytes, &hf));
  IDQ_TRY(data_hvp(ctx, g, dtype, x, y, v, hf, s));
  if (ctx->L == 0 || lambda == 0.0) return copy_state(hf, out, sbytes, s);
  IDQ_TRY(ctx->ws.get(W_HG, sbytes, &hg));
  IDQ_TRY(net_hvp(ctx, g, prec, x, v, hg, s));
  return launch_axpbypcz(1.0, hf, lambda, hg, 0.0, nullptr, out, g.n * g.per, dtype, s);
}

int dot(idq_ctx* ctx, const void* a, const void* b, long long count, int dtype, double* out,
        hipStream_t s) {
  void* part;
  IDQ_TRY(ctx->ws.get(W_PART, 1024 * 8, &part));
  return launch_dot(a, b, count, dtype, static_cast<double*>(part), 1024, out, s);
}

int power_iteration(idq_ctx* ctx, const Geometry& g, int dtype, int prec, const void* x,
                    const void* y, const void* v0, double lambda, int iters, double* L,
                    hipStream_t s) {
  const size_t sbytes = static_cast<size_t>(g.n) * g.per * elem_size(dtype);
  const long long cnt = g.n * g.per;
  void *v, *w, *scal;
  IDQ_TRY(ctx->ws.get(W_V, sbytes, &v));
  IDQ_TRY(ctx->ws.get(W_W, sbytes, &w));
  IDQ_TRY(ctx->ws.get(W_SCAL, 64, &scal));
  double* sc = static_cast<double*>(scal);
  IDQ_TRY(dot(ctx, v0, v0, cnt, dtype, sc, s));
  IDQ_TRY(launch_scale_by(v0, v, cnt, sc, 1, dtype, s));
  for (int it = 0; it < iters; ++it) {
    IDQ_TRY(obj_hvp(ctx, g, dtype, prec, x, y, v, lambda, w, s));
    IDQ_TRY(dot(ctx, v, w, cnt, dtype, sc + 1, s));
    IDQ_TRY(dot(ctx, w, w, cnt, dtype, sc, s));
    IDQ_TRY(launch_scale_by(w, v, cnt, sc, 1, dtype, s));
  }
  double hL = 0.0;
  IDQ_HIP(hipMemcpyAsync(&hL, sc + 1, 8, hipMemcpyDeviceToHost, s));
  IDQ_HIP(hipStreamSynchronize(s));
  *L = hL;
  return IDQ_OK;
}

int ensure_host_gate(idq_ctx* ctx, int n) {
  if (ctx->host_gate_cap < n) {
    if (ctx->host_gate) (void)hipHostFree(ctx->host_gate);
    ctx->host_gate = nullptr;
    IDQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&ctx->host_gate), sizeof(int) * n));
    ctx->host_gate_cap = n;
  }
  return IDQ_OK;
}

}  // namespace

int ws_forward_internal(idq_ws* ws, const void* y, void* x0, int n, int c, int h, int w, int prec,
                        hipStream_t s);  // ws.hip

// The context's stream for graph capture and replay (non-blocking, default
// priority) and its two ordering events, created on first use.
int graph_stream(idq_ctx* ctx, hipStream_t* out) {
  if (!ctx->gstream) {
    IDQ_HIP(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
    IDQ_HIP(hipEventCreateWithFlags(&ctx->gev[0], hipEventDisableTiming));
    IDQ_HIP(hipEventCreateWithFlags(&ctx->gev[1], hipEventDisableTiming));
  }
  *out = ctx->gstream;
  return IDQ_OK;
}

namespace {

int solve_impl(idq_ctx* ctx, const void* y, const void* x0, void* x_out, int n, int c, int h,
               int w, int dtype, const idq_solve_opts* o, idq_solve_info* info, hipStream_t s) {
  if (!y || !x_out || !o || !info) return fail(IDQ_E_INVAL, "null argument");
  Geometry g;
  IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
  IDQ_TRY(check_prec(dtype, o->conv_prec));
  if (o->conv_prec == IDQ_BF16 && o->refine_prec != IDQ_F32 && o->refine_prec != IDQ_BF16X3)
    return fail(IDQ_E_INVAL, "refine_prec must be IDQ_F32 or IDQ_BF16X3");
  if (o->max_iter <= 0 && o->fixed_iters <= 0) return fail(IDQ_E_INVAL, "max_iter must be positive");
  const bool proximal = o->proximal != 0;
  if (proximal && !has_prox(ctx->op_kind))
    return fail(IDQ_E_UNSUPPORTED, "i-DEQ-P needs a data term with a closed-form proximal step");
  if (proximal && o->grad_at != IDQ_GRAD_AT_EXTRAPOLATED)
    return fail(IDQ_E_UNSUPPORTED, "i-DEQ-P evaluates the gradient at the extrapolated point");
  const bool averaging = o->averaging != 0;
  if (averaging && (o->fixed_iters <= 0 || o->restart_B > 0.0 || o->conv_prec == IDQ_BF16))
    return fail(IDQ_E_UNSUPPORTED,
                "averaging needs fixed_iters > 0, restart off and a single conv arithmetic");
  const bool use_net = ctx->L > 0 && o->lambda != 0.0;
  const size_t es = elem_size(dtype);
  const size_t sbytes = static_cast<size_t>(n) * g.per * es;
  const long long cnt = n * g.per;
  void *xb[2], *z, *gf, *q, *part, *state, *gate, *beta;
  IDQ_TRY(ctx->ws.get(W_X0, sbytes, &xb[0]));
  IDQ_TRY(ctx->ws.get(W_X1, sbytes, &xb[1]));
  IDQ_TRY(ctx->ws.get(W_Z, sbytes, &z));
  IDQ_TRY(ctx->ws.get(W_GF, sbytes, &gf));
  IDQ_TRY(ctx->ws.get(W_Q, sbytes, &q));
  const int nblk = static_cast<int>(std::min<long long>(64, (g.per + 4095) / 4096));
  IDQ_TRY(ctx->ws.get(W_PART, static_cast<size_t>(n) * nblk * 3 * 8 + 1024 * 8, &part));
  IDQ_TRY(ctx->ws.get(W_STATE, sizeof(ImgState) * n, &state));
  IDQ_TRY(ctx->ws.get(W_GATE, sizeof(int) * n, &gate));
  IDQ_TRY(ctx->ws.get(W_BETA, sizeof(double) * n, &beta));
  void* hist = nullptr;
  const int hist_len = (o->rel_history && o->history_len > 0) ? o->history_len : 0;
  if (hist_len) {
    IDQ_TRY(ctx->ws.get(W_HIST, sizeof(double) * n * hist_len, &hist));
    std::vector<double> nan(static_cast<size_t>(n) * hist_len, NAN);
    IDQ_HIP(hipMemcpyAsync(hist, nan.data(), sizeof(double) * nan.size(), hipMemcpyHostToDevice, s));
    IDQ_HIP(hipStreamSynchronize(s));
  }
  // A^T y, once per solve, where the steps use it: the MRI gradient
  // F^H M_s F z - A^T y and the Fourier proximal steps
  const bool mri = ctx->op_kind == IDQ_OP_MRI;
  void* aty = nullptr;
  if (mri || (proximal && ctx->op_kind == IDQ_OP_BLUR_CIRC))
    IDQ_TRY(data_aty(ctx, g, dtype, y, &aty, s));
  void* pbuf = nullptr;
  if (proximal) IDQ_TRY(ctx->ws.get(W_PROX, sbytes, &pbuf));
  // x^0 and x^{-1} = x^0
  if (x0) {
    IDQ_TRY(copy_state(x0, xb[0], sbytes, s));
  } else if (o->init == IDQ_INIT_Y && mri) {
    // k-space data: start from the zero-filled image A^T y
    IDQ_TRY(copy_state(aty, xb[0], sbytes, s));
  } else if (o->init == IDQ_INIT_Y) {
    IDQ_TRY(copy_state(y, xb[0], sbytes, s));
  } else if (o->init == IDQ_INIT_ZERO) {
    IDQ_HIP(hipMemsetAsync(xb[0], 0, sbytes, s));
  } else if (o->init == IDQ_INIT_WARMSTART) {
    if (!o->ws || dtype != IDQ_F32 || mri)
      return fail(IDQ_E_INVAL, "warm start needs a network, float32 and image-domain data");
    IDQ_TRY(profiled(ctx, PC_WARMSTART, s, [&] {
      return ws_forward_internal(o->ws, y, xb[0], n, c, h, w, o->ws_prec, s);
    }));
  } else {
    return fail(IDQ_E_INVAL, "bad init");
  }
  if (o->x_prev)
    IDQ_TRY(copy_state(o->x_prev, xb[1], sbytes, s));
  else
    IDQ_TRY(copy_state(xb[0], xb[1], sbytes, s));
  // averaging: running float64 sum of the z^k and the averaged output (x^0
  // until the window's first step)
  double* zsum = nullptr;
  void* xhat = nullptr;
  if (averaging) {
    void* zs;
    IDQ_TRY(ctx->ws.get(W_ZSUM, static_cast<size_t>(cnt) * sizeof(double), &zs));
    IDQ_TRY(ctx->ws.get(W_XHAT, sbytes, &xhat));
    zsum = static_cast<double*>(zs);
    IDQ_HIP(hipMemsetAsync(zsum, 0, static_cast<size_t>(cnt) * sizeof(double), s));
    IDQ_TRY(copy_state(xb[0], xhat, sbytes, s));
  }
  // step size
  double tau = o->tau;
  if (tau <= 0.0) {
    if (!o->power_v0) return fail(IDQ_E_INVAL, "tau == 0 needs power_v0");
    const int pprec = (o->conv_prec == IDQ_BF16 || o->conv_prec == IDQ_BF16X3) ? IDQ_F32
                                                                               : o->conv_prec;
    double L = 0.0;
    IDQ_TRY(power_iteration(ctx, g, dtype, pprec, xb[0], y, o->power_v0, o->lambda,
                            o->power_iters > 0 ? o->power_iters : 30, &L, s));
    if (!(L > 0.0)) return fail(IDQ_E_NONFINITE, "power iteration gave a non-positive L");
    tau = 0.9 / L;
  }
  // per-image state
  const int first_gate = o->conv_prec == IDQ_BF16 ? G_LOW : G_FINAL;
  std::vector<ImgState> hs(n);
  for (auto& st : hs) {
    std::memset(&st, 0, sizeof(st));
    st.status = IDQ_ST_MAXITER;
    st.prec = first_gate;
    st.rel = INFINITY;
    st.best_rel = INFINITY;
    st.avg_best = INFINITY;
  }
  std::vector<int> hg(n, first_gate);
  std::vector<double> hb(n, o->x_prev ? o->beta : 0.0);  // x^{-1} = x^0: no first inertia
  IDQ_HIP(hipMemcpyAsync(state, hs.data(), sizeof(ImgState) * n, hipMemcpyHostToDevice, s));
  IDQ_HIP(hipMemcpyAsync(gate, hg.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  IDQ_HIP(hipMemcpyAsync(beta, hb.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  IDQ_TRY(ensure_host_gate(ctx, n));

  const int limit = o->fixed_iters > 0 ? o->fixed_iters : o->max_iter;
  const int poll = o->poll_every > 0 ? o->poll_every : 8;
  // bf16 start: bf16 -> [split-bf16 if refine_prec says so] -> float32
  const bool bf_start = o->conv_prec == IDQ_BF16;
  const bool use_mid = bf_start && o->refine_prec == IDQ_BF16X3;
  const int final_prec = bf_start ? IDQ_F32 : o->conv_prec;
  // Phases launched in a step, from the last poll: an image moves at most one
  // phase per update, so the bf16 phase ends once a poll finds none in it, and
  // the split phase cannot be reached in the first step after a poll that found
  // none there.  The float32 phase of a bf16 start is launched only once a poll
  // has found an image in it: one that enters it between polls waits, unchanged
  // and uncounted, until then (each image needs about one float32 update, and
  // an empty float32 pass per step costs more than that wait).
  bool low_live = bf_start, mid_live = use_mid, mid_seen = false, fin_live = !bf_start;
  // waiting steps do not count towards an image's iterations
  const int host_limit = bf_start ? limit + 2 * poll + 2 : limit;
  const int* gp = static_cast<const int*>(gate);
  const bool identity = ctx->op_kind == IDQ_OP_IDENTITY;

  FinalizeArgs fa{};
  fa.n = n;
  fa.nblk = nblk;
  fa.partials = static_cast<double*>(part);
  fa.st = static_cast<ImgState*>(state);
  fa.gate = static_cast<int*>(gate);
  fa.beta_eff = static_cast<double*>(beta);
  fa.beta = o->beta;
  fa.tol = o->tol;
  fa.restart_B2 = o->restart_B > 0.0 ? o->restart_B * o->restart_B : 0.0;
  fa.switch_tol = o->switch_tol;
  fa.switch_patience = o->switch_patience > 0 ? o->switch_patience : 10;
  fa.max_iter = o->max_iter;
  fa.fixed_iters = o->fixed_iters;
  fa.use_mid = use_mid ? 1 : 0;
  fa.avg_K = averaging ? o->fixed_iters : 0;
  fa.diverge_ratio = o->diverge_ratio;

  // one solver step t on stream st: extrapolation, gradients, update, finalize
  auto step = [&](int t, int run, bool mid_now, hipStream_t st) -> int {
    void* xa = xb[t % 2];
    void* xp = xb[(t + 1) % 2];
    IDQ_TRY(profiled(ctx, PC_UPDATE, st, [&] {
      return launch_extrap(xa, xp, z, static_cast<const double*>(beta), gp, run, n, g.per,
                           dtype, st);
    }));
    const void* p = o->grad_at == IDQ_GRAD_AT_CURRENT ? xa : z;
    if (!identity && !proximal)
      IDQ_TRY(data_grad(ctx, g, dtype, p, y, gf, gp, st, false, run, aty));
    if (use_net) {
      if (run & (1 << G_LOW)) IDQ_TRY(net_grad(ctx, g, IDQ_BF16, p, q, gp, 1 << G_LOW, st));
      if (mid_now) IDQ_TRY(net_grad(ctx, g, IDQ_BF16X3, p, q, gp, 1 << G_MID, st));
      if (run & (1 << G_FINAL)) IDQ_TRY(net_grad(ctx, g, final_prec, p, q, gp, 1 << G_FINAL, st));
    }
    UpdateArgs ua{};
    ua.n = n;
    ua.per = g.per;
    ua.x = xa;
    ua.xn = xp;
    if (proximal) {
      // i-DEQ-P (Alg. 2): x^{k+1} = prox_{tau f}(z - tau lambda grad g(z)), formed
      // over the whole batch; the update kernel takes it for the images it runs
      IDQ_TRY(profiled(ctx, PC_STENCIL, st, [&] {
        return prox_apply(ctx, g, dtype, z, use_net ? q : nullptr, -tau * o->lambda, y, aty, tau,
                          pbuf, st);
      }));
      ua.z = pbuf;
      ua.given = 1;
    } else {
      ua.z = z;
      ua.gf = identity ? nullptr : gf;
      ua.p = p;
      ua.y = y;
      ua.q = use_net ? q : nullptr;
    }
    ua.tau = tau;
    ua.lambda = o->lambda;
    ua.gate = gp;
    ua.run_mask = run;
    ua.partials = static_cast<double*>(part);
    ua.nblk = nblk;
    FinalizeArgs fs = fa;
    fs.buf_index = (t + 1) % 2;
    fs.history = static_cast<double*>(hist);
    fs.history_rows = hist_len;
    fs.run_mask = run;
    IDQ_TRY(profiled(ctx, PC_UPDATE, st, [&] {
      IDQ_TRY(launch_update(ua, dtype, st));
      return launch_finalize(fs, st);
    }));
    // with averaging every image updates on every step, so step t is update t + 1
    if (averaging)
      IDQ_TRY(launch_average(z, zsum, xhat, static_cast<const ImgState*>(state), t + 1, n, g.per,
                             dtype, st));
    return IDQ_OK;
  };

  int t = 0;
  // A fixed number of steps in one arithmetic needs no host decision between
  // them: step 0 runs as usual (it sizes every workspace buffer), steps 1 and 2
  // are captured into a HIP graph once, and the graph is replayed for each
  // following pair (the buffers' roles repeat with period 2).  Launch-bound
  // solves (small images) then pay one graph launch per two steps.
  if (o->use_graph && !bf_start && !ctx->prof.on && !averaging && o->fixed_iters >= 3) {
    const int run = 1 << G_FINAL;
    IDQ_TRY(step(0, run, false, s));
    hipStream_t gs;
    IDQ_TRY(graph_stream(ctx, &gs));
    IDQ_HIP(hipEventRecord(ctx->gev[0], s));
    IDQ_HIP(hipStreamWaitEvent(gs, ctx->gev[0], 0));
    const int pairs = (limit - 1) / 2;
    hipGraph_t graph = nullptr;
    IDQ_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed));
    int rc1 = step(1, run, false, gs);
    int rc2 = rc1 < 0 ? rc1 : step(2, run, false, gs);
    hipError_t ec = hipStreamEndCapture(gs, &graph);
    if (rc2 < 0) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc2;
    }
    if (ec != hipSuccess) return fail(IDQ_E_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ec != hipSuccess) return fail(IDQ_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ec));
    for (int pr = 0; pr < pairs && ec == hipSuccess; ++pr) ec = hipGraphLaunch(exec, gs);
    t = 1 + 2 * pairs;
    int rc3 = (ec == hipSuccess && t < limit) ? step(t, run, false, gs) : IDQ_OK;
    hipError_t es = hipStreamSynchronize(gs);
    (void)hipGraphExecDestroy(exec);
    if (ec != hipSuccess) return fail(IDQ_E_HIP, std::string("graph launch: ") + hipGetErrorString(ec));
    if (es != hipSuccess) return fail(IDQ_E_HIP, std::string("graph stream: ") + hipGetErrorString(es));
    IDQ_TRY(rc3);
    t = host_limit;
  }
  while (t < host_limit) {
    // once only float32-phase images remain (a bf16 start), each needs about one
    // more update: poll after every step rather than launch empty steps
    const bool fin_only = bf_start && fin_live && !low_live && !mid_live;
    const int t_end = std::min(host_limit, t + (fin_only ? 1 : poll));
    for (int j = 0; t < t_end; ++t, ++j) {
      const bool mid_now = mid_live && (j > 0 || mid_seen);
      const int run = (low_live ? 1 << G_LOW : 0) | (mid_now ? 1 << G_MID : 0) |
                      (fin_live ? 1 << G_FINAL : 0);
      IDQ_TRY(step(t, run, mid_now, s));
    }
    IDQ_HIP(hipMemcpyAsync(ctx->host_gate, gate, sizeof(int) * n, hipMemcpyDeviceToHost, s));
    IDQ_HIP(hipStreamSynchronize(s));
    if (ctx->prof.on) IDQ_TRY(ctx->prof.flush());
    bool any = false, anylow = false, anymid = false, anyfin = false;
    for (int i = 0; i < n; ++i) {
      any |= ctx->host_gate[i] != G_DONE;
      anylow |= ctx->host_gate[i] == G_LOW;
      anymid |= ctx->host_gate[i] == G_MID;
      anyfin |= ctx->host_gate[i] == G_FINAL;
    }
    low_live = anylow;
    mid_live = use_mid && (anylow || anymid);
    mid_seen = anymid;
    fin_live = !bf_start || anyfin;
    if (!any) break;
  }
  if (averaging)
    IDQ_TRY(copy_state(xhat, x_out, sbytes, s));
  else
    IDQ_TRY(launch_gather_result(xb[0], xb[1], x_out, static_cast<const ImgState*>(state), n,
                                 g.per, dtype, s));
  if (o->x_prev_out)
    IDQ_TRY(launch_gather_result(xb[0], xb[1], o->x_prev_out, static_cast<const ImgState*>(state),
                                 n, g.per, dtype, s, 1));
  IDQ_HIP(hipMemcpyAsync(hs.data(), state, sizeof(ImgState) * n, hipMemcpyDeviceToHost, s));
  if (hist_len)
    IDQ_HIP(hipMemcpyAsync(o->rel_history, hist, sizeof(double) * n * hist_len,
                           hipMemcpyDeviceToHost, s));
  IDQ_HIP(hipStreamSynchronize(s));
  int rc = IDQ_OK;
  for (int i = 0; i < n; ++i) {
    info[i].iters = hs[i].it;
    info[i].iters_low = hs[i].it_low;
    info[i].iters_mid = hs[i].it_mid;
    info[i].restarts = hs[i].restarts;
    info[i].status = hs[i].status;
    info[i].rel = hs[i].rel;
    info[i].tau = tau;
    if (hs[i].status == IDQ_ST_NONFINITE) {
      if (rc != IDQ_E_NONFINITE)
        set_error("image " + std::to_string(i) + " produced a non-finite iterate after " +
                  std::to_string(hs[i].it) + " updates");
      rc = IDQ_E_NONFINITE;
    } else if (hs[i].status == IDQ_ST_DIVERGED) {
      if (rc >= 0)
        set_error("image " + std::to_string(i) + " diverged: its iterate norm passed " +
                  std::to_string(o->diverge_ratio) + " times the initial one after " +
                  std::to_string(hs[i].it) + " updates");
      if (rc >= 0) rc = IDQ_E_DIVERGED;
    } else if (hs[i].status == IDQ_ST_MAXITER && rc == IDQ_OK) {
      set_error("image " + std::to_string(i) + " reached max_iter");
      rc = IDQ_W_MAXITER;
    }
  }
  (void)cnt;
  return rc;
}

int backward_impl(idq_ctx* ctx, const void* xbar, const void* y, const void* v, void* dtheta,
                  double* dlambda, int n, int c, int h, int w, int dtype, const idq_bwd_opts* o,
                  idq_bwd_info* info, hipStream_t s) {
  if (!xbar || !y || !v || !dtheta || !o) return fail(IDQ_E_INVAL, "null argument");
  if (ctx->L == 0) return fail(IDQ_E_INVAL, "no network");
  Geometry g;
  IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
  const int prec = dtype;  // the backward runs in the tensors' own arithmetic
  IDQ_TRY(check_prec(dtype, prec));
  const size_t sbytes = static_cast<size_t>(n) * g.per * elem_size(dtype);
  const long long cnt = n * g.per;
  void *u, *up, *un, *hw, *scal;
  IDQ_TRY(ctx->ws.get(W_U, sbytes, &u));
  IDQ_TRY(ctx->ws.get(W_UP, sbytes, &up));
  IDQ_TRY(ctx->ws.get(W_UN, sbytes, &un));
  IDQ_TRY(ctx->ws.get(W_W, sbytes, &hw));
  IDQ_TRY(ctx->ws.get(W_SCAL, 64, &scal));
  double* sc = static_cast<double*>(scal);
  const bool proximal = o->proximal != 0;
  if (proximal && !has_prox(ctx->op_kind))
    return fail(IDQ_E_UNSUPPORTED, "i-DEQ-P needs a data term with a closed-form proximal step");
  // J_P w = (I + tau A^T A)^{-1} w, the Jacobian of the proximal step: the
  // proximal step with y = 0
  void* zero = nullptr;
  if (proximal) {
    const size_t ybytes = sbytes * (ctx->op_kind == IDQ_OP_MRI ? 2 : 1);
    IDQ_TRY(ctx->ws.get(W_PROX, ybytes, &zero));
    IDQ_HIP(hipMemsetAsync(zero, 0, ybytes, s));
  }
  auto prox_lin = [&](const void* in, void* out) {
    return prox_apply(ctx, g, dtype, in, nullptr, 0.0, zero, zero, o->tau, out, s);
  };
  IDQ_TRY(copy_state(v, u, sbytes, s));
  int iters = 0;
  double rel = 0.0;
  if (o->mode == IDQ_BWD_IMPLICIT) {
    IDQ_TRY(copy_state(v, up, sbytes, s));
    void *wv, *pw = nullptr;
    IDQ_TRY(ctx->ws.get(W_V, sbytes, &wv));
    if (proximal) IDQ_TRY(ctx->ws.get(W_PW, sbytes, &pw));
    // the relative change of each iteration goes to a device slot; the host
    // reads them every kCheck iterations (and at the last), and the iteration
    // that first met the tolerance ends the loop at the next check
    constexpr int kCheck = 8;
    void* relbuf;
    IDQ_TRY(ctx->ws.get(W_HIST, sizeof(double) * 2 * kCheck, &relbuf));
    double* rb = static_cast<double*>(relbuf);
    for (int j = 1; j <= o->adjoint_max_iter; ++j) {
      // w = u + beta (u - up)
      IDQ_TRY(launch_axpbypcz(1.0 + o->adjoint_beta, u, -o->adjoint_beta, up, 0.0, nullptr, wv, cnt,
                              dtype, s));
      if (!proximal) {
        // un = w - tau H_F w + v
        IDQ_TRY(obj_hvp(ctx, g, dtype, prec, xbar, y, wv, o->lambda, hw, s));
        IDQ_TRY(launch_axpbypcz(1.0, wv, -o->tau, hw, 1.0, v, un, cnt, dtype, s));
      } else {
        // un = J_P w - tau lambda H_g J_P w + v
        IDQ_TRY(prox_lin(wv, pw));
        IDQ_TRY(net_hvp(ctx, g, prec, xbar, pw, hw, s));
        IDQ_TRY(launch_axpbypcz(1.0, pw, -o->tau * o->lambda, hw, 1.0, v, un, cnt, dtype, s));
      }
      // rel = ||un - u|| / ||u||
      const int slot = (j - 1) % kCheck;
      IDQ_TRY(launch_axpbypcz(1.0, un, -1.0, u, 0.0, nullptr, up, cnt, dtype, s));
      IDQ_TRY(dot(ctx, up, up, cnt, dtype, rb + 2 * slot, s));
      IDQ_TRY(dot(ctx, u, u, cnt, dtype, rb + 2 * slot + 1, s));
      // rotate: up <- u, u <- un
      void* tmp = up;
      up = u;
      u = un;
      un = tmp;
      iters = j;
      if (slot == kCheck - 1 || j == o->adjoint_max_iter) {
        double hsc[2 * kCheck];
        IDQ_HIP(hipMemcpyAsync(hsc, rb, sizeof(double) * 2 * (slot + 1), hipMemcpyDeviceToHost, s));
        IDQ_HIP(hipStreamSynchronize(s));
        bool met = false;
        for (int q = 0; q <= slot; ++q) {
          rel = std::sqrt(hsc[2 * q] / std::max(hsc[2 * q + 1], 1e-300));
          if (!(rel >= o->adjoint_tol)) met = true;
        }
        if (met) break;
      }
    }
  }
  // the vector the parameter gradient uses: u, or J_P u for i-DEQ-P
  if (proximal) {
    IDQ_TRY(prox_lin(u, un));
    u = un;
  }
  // theta gradient from the forward-over-reverse pass along u
  void* hgout;
  IDQ_TRY(ctx->ws.get(W_HG, sbytes, &hgout));
  IDQ_TRY(net_hvp(ctx, g, prec, xbar, u, hgout, s));
  const double scale = o->tau * o->lambda;
  const size_t abytes = static_cast<size_t>(g.pix()) * max_ch(ctx) * act_size(prec);
  const long long pix = g.pix();
  const int nchunk = static_cast<int>(std::max<long long>(1, std::min<long long>(256, pix / 1024)));
  size_t off = 0;
  for (int l = 0; l < ctx->L; ++l) {
    const int ci = ctx->ch[l], co = ctx->ch[l + 1];
    const int nslots = co * ci * 9 + co;
    void* wgp;
    IDQ_TRY(ctx->ws.get(W_WGPART, static_cast<size_t>(nchunk) * nslots * 8, &wgp));
    void *gdd, *gd, *a0, *a1, *hprev = nullptr, *hdprev = nullptr;
    if (l == ctx->L - 1) {
      IDQ_TRY(ctx->ws.get(W_RD, sbytes, &gdd));
      IDQ_TRY(ctx->ws.get(W_R, sbytes, &gd));
    } else {
      IDQ_TRY(ctx->ws.get(W_DDL0 + l, abytes, &gdd));
      IDQ_TRY(ctx->ws.get(W_DL0 + l, abytes, &gd));
    }
    if (l > 0) {
      IDQ_TRY(ctx->ws.get(W_H0 + l - 1, abytes, &hprev));
      IDQ_TRY(ctx->ws.get(W_HD0 + l - 1, abytes, &hdprev));
    }
    const int gfmt = l == ctx->L - 1 ? F_NCHW : F_NHWC;
    WgradArgs wa{};
    wa.NI = g.NI;
    wa.H = g.h;
    wa.W = g.w;
    wa.CI = ci;
    wa.CO = co;
    wa.g_fmt = gfmt;
    wa.act = ctx->act;
    wa.partials = static_cast<double*>(wgp);
    wa.nchunk = nchunk;
    // delta'_l corr a_{l-1}  (+ bias: sum delta'_l)
    wa.g = gdd;
    if (l == 0) {
      wa.a_fmt = F_NCHW;
      wa.a_pro = P_NONE;
      wa.a0 = xbar;
    } else {
      wa.a_fmt = F_NHWC;
      wa.a_pro = P_NONE;
      wa.a0 = hprev;
    }
    wa.with_bias = 1;
    IDQ_TRY(launch_wgrad(wa, prec, s));
    char* dst = static_cast<char*>(dtheta) + off * elem_size(dtype);
    IDQ_TRY(launch_reduce_chunks(static_cast<double*>(wgp), nchunk, nslots, scale, dst, 0, dtype, s));
    // delta_l corr a'_{l-1}
    wa.g = gd;
    if (l == 0) {
      wa.a0 = u;
      wa.a_pro = P_NONE;
    } else {
      wa.a0 = hprev;
      wa.a1 = hdprev;
      wa.a_pro = P_JVP;
    }
    wa.with_bias = 0;
    IDQ_TRY(launch_wgrad(wa, prec, s));
    IDQ_TRY(launch_reduce_chunks(static_cast<double*>(wgp), nchunk, co * ci * 9, scale, dst, 1,
                                 dtype, s));
    off += static_cast<size_t>(nslots);
  }
  // dlambda = -tau <grad g(xbar), u>
  if (dlambda) {
    void* q;
    IDQ_TRY(ctx->ws.get(W_Q, sbytes, &q));
    IDQ_TRY(net_grad(ctx, g, prec, xbar, q, nullptr, 0, s));
    IDQ_TRY(dot(ctx, q, u, cnt, dtype, sc + 2, s));
    double d = 0.0;
    IDQ_HIP(hipMemcpyAsync(&d, sc + 2, 8, hipMemcpyDeviceToHost, s));
    IDQ_HIP(hipStreamSynchronize(s));
    *dlambda = -o->tau * d;
  }
  IDQ_HIP(hipStreamSynchronize(s));
  if (info) {
    info->adjoint_iters = iters;
    info->adjoint_rel = rel;
  }
  return IDQ_OK;
}

void free_operator(idq_ctx* ctx) {
  for (int d = 0; d < 2; ++d)
    for (void** q : {&ctx->mask_dev[d], &ctx->msym_dev[d], &ctx->spec_dev[d]})
      if (*q) {
        (void)hipFree(*q);
        *q = nullptr;
      }
}

// Copies the 0/1 mask of an inpainting or MRI operator to the device in float64
// and float32; for MRI also M_s(k) = (M(k) + M(-k)) / 2 (-k taken mod h, w),
// the multiplier of A^T A = Re(F^H M F) on real images.
int upload_mask(idq_ctx* ctx, const idq_op_desc* op) {
  if (!op->mask || op->mh <= 0 || op->mw <= 0)
    return fail(IDQ_E_INVAL, "mask operators need a mask and its size");
  const int h = op->mh, w = op->mw;
  const size_t cnt = static_cast<size_t>(h) * w;
  for (size_t i = 0; i < cnt; ++i)
    if (op->mask[i] != 0.0 && op->mask[i] != 1.0) return fail(IDQ_E_INVAL, "mask values must be 0 or 1");
  if (op->kind == IDQ_OP_MRI && !fft_supported(h, w))
    return fail(IDQ_E_UNSUPPORTED, "the MRI operator needs power-of-two h and w in [4, 1024]");
  ctx->mh = h;
  ctx->mw = w;
  std::vector<double> sym(cnt);
  for (int i = 0; i < h; ++i)
    for (int j = 0; j < w; ++j)
      sym[static_cast<size_t>(i) * w + j] =
          0.5 * (op->mask[static_cast<size_t>(i) * w + j] +
                 op->mask[static_cast<size_t>((h - i) % h) * w + (w - j) % w]);
  std::vector<float> mf(op->mask, op->mask + cnt), sf(sym.begin(), sym.end());
  IDQ_TRY(upload(&ctx->mask_dev[0], op->mask, cnt * 8));
  IDQ_TRY(upload(&ctx->mask_dev[1], mf.data(), cnt * 4));
  if (op->kind == IDQ_OP_MRI) {
    IDQ_TRY(upload(&ctx->msym_dev[0], sym.data(), cnt * 8));
    IDQ_TRY(upload(&ctx->msym_dev[1], sf.data(), cnt * 4));
  }
  return IDQ_OK;
}

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(IDQ_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(IDQ_E_INVAL, e.what());
  } catch (...) {
    return fail(IDQ_E_INVAL, "unknown exception");
  }
}

int set_device(const idq_ctx* ctx) {
  IDQ_HIP(hipSetDevice(ctx->device));
  return IDQ_OK;
}

}  // namespace
}  // namespace idq

namespace idq {
// Entry points of the training loop (train.hip) into the solver and the backward.
int solve_internal(idq_ctx* ctx, const void* y, const void* x0, void* x_out, int n, int c, int h,
                   int w, int dtype, const idq_solve_opts* o, idq_solve_info* info,
                   hipStream_t s) {
  return solve_impl(ctx, y, x0, x_out, n, c, h, w, dtype, o, info, s);
}
int backward_internal(idq_ctx* ctx, const void* xbar, const void* y, const void* v, void* dtheta,
                      double* dlambda, int n, int c, int h, int w, int dtype,
                      const idq_bwd_opts* o, idq_bwd_info* info, hipStream_t s) {
  return backward_impl(ctx, xbar, y, v, dtheta, dlambda, n, c, h, w, dtype, o, info, s);
}
int repack_weights(idq_ctx* ctx) { return pack_weights(ctx); }
int dot_batch(idq_ctx* ctx, const void* a, const void* b, long long count, int dtype, double* out,
              hipStream_t s) {
  return dot(ctx, a, b, count, dtype, out, s);
}
}  // namespace idq

using namespace idq;

extern "C" {

const char* idq_last_error(void) { return g_err.c_str(); }
int idq_version(void) { return 10000; }

void idq_solve_opts_default(idq_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->beta = 0.5;
  o->tau = 0.0;
  o->lambda = 1.0;
  o->tol = 1e-4;
  o->max_iter = 1000;
  o->fixed_iters = 0;
  o->restart_B = 0.0;
  o->grad_at = IDQ_GRAD_AT_EXTRAPOLATED;
  o->conv_prec = IDQ_F32;
  o->switch_tol = 2e-3;
  o->switch_patience = 5;
  o->power_iters = 30;
  o->poll_every = 8;
  o->init = IDQ_INIT_Y;
  o->ws_prec = IDQ_BF16;
  o->refine_prec = IDQ_F32;
  o->use_graph = 1;
  o->diverge_ratio = 1e6;
}

int idq_create(idq_ctx** out, const idq_net_desc* net, const idq_op_desc* op, int device) {
  return guarded([&]() -> int {
    if (!out || !op) return fail(IDQ_E_INVAL, "null argument");
    *out = nullptr;
    int ndev = 0;
    IDQ_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(IDQ_E_INVAL, "bad device index");
    IDQ_HIP(hipSetDevice(device));
    // the allocation-free entry points' scratch address on this device
    IDQ_TRY(noalloc_init_device(device));
    auto* ctx = new idq_ctx();
    ctx->device = device;
    if (net && net->n_layers > 0) {
      if (net->n_layers > IDQ_MAX_LAYERS || !net->params) {
        delete ctx;
        return fail(IDQ_E_INVAL, "bad network description");
      }
      ctx->L = net->n_layers;
      ctx->act = net->act;
      if (net->act != IDQ_ACT_SOFTPLUS && net->act != IDQ_ACT_IDENTITY) {
        delete ctx;
        return fail(IDQ_E_INVAL, "bad activation");
      }
      size_t total = 0;
      for (int l = 0; l <= ctx->L; ++l) {
        ctx->ch[l] = net->channels[l];
        if (ctx->ch[l] <= 0 || ctx->ch[l] > 1024) {
          delete ctx;
          return fail(IDQ_E_INVAL, "bad channel count");
        }
      }
      if (ctx->ch[0] != ctx->ch[ctx->L]) {
        delete ctx;
        return fail(IDQ_E_INVAL, "network must map c channels to c channels");
      }
      for (int l = 0; l < ctx->L; ++l)
        total += static_cast<size_t>(ctx->ch[l + 1]) * ctx->ch[l] * 9 + ctx->ch[l + 1];
      ctx->params.assign(net->params, net->params + total);
    }
    ctx->op_kind = op->kind;
    if (op->kind == IDQ_OP_INPAINT || op->kind == IDQ_OP_MRI) {
      int rc = upload_mask(ctx, op);
      if (rc < 0) {
        free_operator(ctx);
        delete ctx;
        return rc;
      }
    } else if (op->kind == IDQ_OP_RICIAN) {
      if (!(op->sigma > 0.0) || !std::isfinite(op->sigma)) {
        delete ctx;
        return fail(IDQ_E_INVAL, "the Rician term needs sigma > 0");
      }
      ctx->sigma = op->sigma;
    } else if (op->kind != IDQ_OP_IDENTITY) {
      if (op->kind != IDQ_OP_BLUR_CIRC && op->kind != IDQ_OP_TANH_BLUR) {
        delete ctx;
        return fail(IDQ_E_INVAL, "bad operator kind");
      }
      if (!op->taps || op->kh <= 0 || op->kw <= 0 || op->kh % 2 == 0 || op->kw % 2 == 0 ||
          op->kh > 9 || op->kw > 9) {
        delete ctx;
        return fail(IDQ_E_INVAL, "blur taps must be odd-sized, at most 9x9");
      }
      ctx->kh = op->kh;
      ctx->kw = op->kw;
      ctx->taps.assign(op->taps, op->taps + op->kh * op->kw);
      ctx->gain = op->gain;
      if (op->kind == IDQ_OP_TANH_BLUR && !(op->gain > 0.0)) {
        delete ctx;
        return fail(IDQ_E_INVAL, "tanh-blur gain must be positive");
      }
    }
    if (ctx->L > 0) {
      int rc = pack_weights(ctx);
      if (rc < 0) {
        free_layers(ctx);
        free_operator(ctx);
        delete ctx;
        return rc;
      }
    }
    *out = ctx;
    return IDQ_OK;
  });
}

int idq_profile_enable(idq_ctx* ctx, int on) {
  return guarded([&]() -> int {
    if (!ctx) return fail(IDQ_E_INVAL, "null context");
    IDQ_TRY(set_device(ctx));
    IDQ_HIP(hipDeviceSynchronize());
    IDQ_TRY(ctx->prof.flush());
    if (!ctx->prof.dev_px) IDQ_HIP(hipMalloc(&ctx->prof.dev_px, sizeof(unsigned long long) * PC_COUNT));
    IDQ_HIP(hipMemset(ctx->prof.dev_px, 0, sizeof(unsigned long long) * PC_COUNT));
    for (int i = 0; i < PC_COUNT; ++i) {
      ctx->prof.ms[i] = 0.0;
      ctx->prof.launches[i] = 0;
      ctx->prof.seen[i] = 0;
    }
    ctx->prof.on = on != 0;
    ctx->prof.mask = static_cast<unsigned>(on);
    return IDQ_OK;
  });
}

int idq_profile_sample(idq_ctx* ctx, int every) {
  return guarded([&]() -> int {
    if (!ctx || every < 1) return fail(IDQ_E_INVAL, "profile sampling needs every >= 1");
    ctx->prof.every = every;
    for (int i = 0; i < PC_COUNT; ++i) ctx->prof.seen[i] = 0;
    return IDQ_OK;
  });
}

int idq_profile_read(idq_ctx* ctx, int cls, double* total_ms, long long* launches,
                     double* pixels) {
  return guarded([&]() -> int {
    if (!ctx || cls < 0 || cls >= PC_COUNT) return fail(IDQ_E_INVAL, "bad profile class");
    IDQ_TRY(set_device(ctx));
    IDQ_HIP(hipDeviceSynchronize());
    IDQ_TRY(ctx->prof.flush());
    unsigned long long px = 0;
    if (ctx->prof.dev_px)
      IDQ_HIP(hipMemcpy(&px, ctx->prof.dev_px + cls, sizeof(px), hipMemcpyDeviceToHost));
    if (total_ms) *total_ms = ctx->prof.ms[cls];
    if (launches) *launches = ctx->prof.launches[cls];
    if (pixels) *pixels = static_cast<double>(px);
    return IDQ_OK;
  });
}

int idq_destroy(idq_ctx* ctx) {
  if (!ctx) return IDQ_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->prof.release();
  free_layers(ctx);
  free_operator(ctx);
  if (ctx->gstream) {
    (void)hipStreamDestroy(ctx->gstream);
    (void)hipEventDestroy(ctx->gev[0]);
    (void)hipEventDestroy(ctx->gev[1]);
  }
  ctx->ws.release();
  if (ctx->host_gate) (void)hipHostFree(ctx->host_gate);
  delete ctx;
  return IDQ_OK;
}

long long idq_num_params(const idq_ctx* ctx) {
  return ctx ? static_cast<long long>(ctx->params.size()) : 0;
}

int idq_set_params(idq_ctx* ctx, const double* params, long long count) {
  return guarded([&]() -> int {
    if (!ctx || !params) return fail(IDQ_E_INVAL, "null argument");
    if (count != static_cast<long long>(ctx->params.size()))
      return fail(IDQ_E_INVAL, "parameter count mismatch");
    IDQ_TRY(set_device(ctx));
    IDQ_HIP(hipDeviceSynchronize());
    ctx->params.assign(params, params + count);
    return pack_weights(ctx);
  });
}

int idq_apply_A(idq_ctx* ctx, const void* x, void* Ax, int n, int c, int h, int w, int dtype,
                void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !x || !Ax) return fail(IDQ_E_INVAL, "null argument");
    if (dtype != IDQ_F64 && dtype != IDQ_F32) return fail(IDQ_E_INVAL, "bad dtype");
    Geometry g;
    IDQ_TRY(set_device(ctx));
    IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (ctx->op_kind) {
      case IDQ_OP_IDENTITY:
        return copy_state(x, Ax, static_cast<size_t>(n) * g.per * elem_size(dtype), s);
      case IDQ_OP_RICIAN:
        return fail(IDQ_E_UNSUPPORTED, "the Rician model has no forward operator");
      case IDQ_OP_INPAINT:
        return datafit(ctx, g, dtype, D_MASK_APPLY, x, nullptr, nullptr, Ax, 0.0, s);
      case IDQ_OP_MRI:
        return mri_forward(ctx, g, dtype, x, Ax, s);
      default:
        break;
    }
    StencilArgs a = stencil_base(ctx, g, nullptr);
    a.in0 = x;
    a.out = Ax;
    a.mode = ctx->op_kind == IDQ_OP_BLUR_CIRC ? S_B : S_TANH_A;
    return launch_stencil(a, ctx->taps.data(), dtype, s);
  });
}

int idq_apply_AT(idq_ctx* ctx, const void* x, const void* v, void* out, int n, int c, int h,
                 int w, int dtype, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !v || !out) return fail(IDQ_E_INVAL, "null argument");
    if (dtype != IDQ_F64 && dtype != IDQ_F32) return fail(IDQ_E_INVAL, "bad dtype");
    Geometry g;
    IDQ_TRY(set_device(ctx));
    IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t sbytes = static_cast<size_t>(n) * g.per * elem_size(dtype);
    switch (ctx->op_kind) {
      case IDQ_OP_IDENTITY:
        return copy_state(v, out, sbytes, s);
      case IDQ_OP_RICIAN:
        return fail(IDQ_E_UNSUPPORTED, "the Rician model has no forward operator");
      case IDQ_OP_INPAINT:
        return datafit(ctx, g, dtype, D_MASK_APPLY, v, nullptr, nullptr, out, 0.0, s);
      case IDQ_OP_MRI:
        return mri_adjoint(ctx, g, dtype, v, out, s);
      default:
        break;
    }
    const void* src = v;
    if (ctx->op_kind == IDQ_OP_TANH_BLUR) {
      if (!x) return fail(IDQ_E_INVAL, "the tanh-blur adjoint needs the linearisation point x");
      void* tmp;
      IDQ_TRY(ctx->ws.get(W_S, sbytes, &tmp));
      StencilArgs a = stencil_base(ctx, g, nullptr);
      a.in0 = x;
      a.aux = v;
      a.out = tmp;
      a.mode = S_TANH_JTW;
      IDQ_TRY(launch_stencil(a, ctx->taps.data(), dtype, s));
      src = tmp;
    }
    StencilArgs b = stencil_base(ctx, g, nullptr);
    b.in0 = src;
    b.out = out;
    b.mode = S_BT;
    return launch_stencil(b, ctx->taps.data(), dtype, s);
  });
}

int idq_grad_data(idq_ctx* ctx, const void* x, const void* y, void* grad, int n, int c, int h,
                  int w, int dtype, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !x || !y || !grad) return fail(IDQ_E_INVAL, "null argument");
    if (dtype != IDQ_F64 && dtype != IDQ_F32) return fail(IDQ_E_INVAL, "bad dtype");
    Geometry g;
    IDQ_TRY(set_device(ctx));
    IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
    return data_grad(ctx, g, dtype, x, y, grad, nullptr, static_cast<hipStream_t>(stream), true);
  });
}

int idq_grad_reg(idq_ctx* ctx, const void* x, void* grad, double* g_val, int n, int c, int h,
                 int w, int dtype, int conv_prec, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !x || !grad) return fail(IDQ_E_INVAL, "null argument");
    if (ctx->L == 0) return fail(IDQ_E_INVAL, "context has no network");
    IDQ_TRY(check_prec(dtype, conv_prec));
    Geometry g;
    IDQ_TRY(set_device(ctx));
    IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
    hipStream_t s = static_cast<hipStream_t>(stream);
    IDQ_TRY(net_grad(ctx, g, conv_prec, x, grad, nullptr, 0, s));
    if (g_val) {
      void *r, *part, *scal;
      IDQ_TRY(ctx->ws.get(W_R, static_cast<size_t>(n) * g.per * elem_size(dtype), &r));
      IDQ_TRY(ctx->ws.get(W_PART, static_cast<size_t>(n) * 64 * 8 + 1024 * 8, &part));
      IDQ_TRY(ctx->ws.get(W_SCAL, std::max<size_t>(64, sizeof(double) * n), &scal));
      IDQ_TRY(launch_half_sqnorm_per_image(r, n, g.per, dtype, static_cast<double*>(part), 64,
                                           static_cast<double*>(scal), s));
      IDQ_HIP(hipMemcpyAsync(g_val, scal, sizeof(double) * n, hipMemcpyDeviceToHost, s));
      IDQ_HIP(hipStreamSynchronize(s));
    }
    return IDQ_OK;
  });
}

int idq_prox_data(idq_ctx* ctx, const void* v, const void* y, double tau, void* out, int n, int c,
                  int h, int w, int dtype, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !v || !y || !out) return fail(IDQ_E_INVAL, "null argument");
    if (dtype != IDQ_F64 && dtype != IDQ_F32) return fail(IDQ_E_INVAL, "bad dtype");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(IDQ_E_INVAL, "tau must be positive");
    if (!has_prox(ctx->op_kind))
      return fail(IDQ_E_UNSUPPORTED, "this data term has no closed-form proximal step");
    Geometry g;
    IDQ_TRY(set_device(ctx));
    IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* aty = nullptr;
    if (ctx->op_kind == IDQ_OP_BLUR_CIRC || ctx->op_kind == IDQ_OP_MRI)
      IDQ_TRY(data_aty(ctx, g, dtype, y, &aty, s));
    return prox_apply(ctx, g, dtype, v, nullptr, 0.0, y, aty, tau, out, s);
  });
}

int idq_hvp(idq_ctx* ctx, const void* x, const void* y, const void* v, void* out, double lambda,
            int which, int n, int c, int h, int w, int dtype, int conv_prec, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !x || !v || !out) return fail(IDQ_E_INVAL, "null argument");
    IDQ_TRY(check_prec(dtype, conv_prec));
    if (conv_prec == IDQ_BF16 || conv_prec == IDQ_BF16X3)
      return fail(IDQ_E_UNSUPPORTED, "HVP is float32/float64 only");
    Geometry g;
    IDQ_TRY(set_device(ctx));
    IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (which == 0) {
      if (ctx->L == 0) return fail(IDQ_E_INVAL, "context has no network");
      return net_hvp(ctx, g, conv_prec, x, v, out, s);
    }
    if (!y) return fail(IDQ_E_INVAL, "objective HVP needs y");
    return obj_hvp(ctx, g, dtype, conv_prec, x, y, v, lambda, out, s);
  });
}

int idq_lipschitz(idq_ctx* ctx, const void* x, const void* y, const void* v0, double lambda,
                  int iters, int n, int c, int h, int w, int dtype, int conv_prec, double* L) {
  return guarded([&]() -> int {
    if (!ctx || !x || !y || !v0 || !L) return fail(IDQ_E_INVAL, "null argument");
    IDQ_TRY(check_prec(dtype, conv_prec));
    if (conv_prec == IDQ_BF16 || conv_prec == IDQ_BF16X3)
      return fail(IDQ_E_UNSUPPORTED, "HVP is float32/float64 only");
    if (iters <= 0) return fail(IDQ_E_INVAL, "iters must be positive");
    Geometry g;
    IDQ_TRY(set_device(ctx));
    IDQ_TRY(check_shape(ctx, n, c, h, w, &g));
    return power_iteration(ctx, g, dtype, conv_prec, x, y, v0, lambda, iters, L, nullptr);
  });
}

int idq_solve(idq_ctx* ctx, const void* y, const void* x0, void* x_out, int n, int c, int h,
              int w, int dtype, const idq_solve_opts* opts, idq_solve_info* info, void* stream) {
  return guarded([&]() -> int {
    if (!ctx) return fail(IDQ_E_INVAL, "null context");
    IDQ_TRY(set_device(ctx));
    return solve_impl(ctx, y, x0, x_out, n, c, h, w, dtype, opts, info,
                      static_cast<hipStream_t>(stream));
  });
}

int idq_backward(idq_ctx* ctx, const void* xbar, const void* y, const void* dl_dx, void* dtheta,
                 double* dlambda, int n, int c, int h, int w, int dtype, const idq_bwd_opts* opts,
                 idq_bwd_info* info, void* stream) {
  return guarded([&]() -> int {
    if (!ctx) return fail(IDQ_E_INVAL, "null context");
    IDQ_TRY(set_device(ctx));
    return backward_impl(ctx, xbar, y, dl_dx, dtheta, dlambda, n, c, h, w, dtype, opts, info,
                         static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
