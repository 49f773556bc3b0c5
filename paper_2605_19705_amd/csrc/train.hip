// The training loop of Alg. 1 (Alg. 2 for i-DEQ-P): one epoch accumulates the
// gradient of the loss over the dataset, each pair's fixed-point estimate from
// K updates of the i-DEQ iteration and its gradient from the JFB or implicit
// backward (App. D.1), then takes one Adam step on Theta = {theta, lambda}.
// The float64 master parameters, the Adam moments and the gradient accumulator
// live on the device; after each step theta is copied back into the context,
// which packs it for every conv arithmetic.
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"

struct idq_trainer {
  idq_ctx* ctx = nullptr;
  long long P = 0;           // network parameters; index P holds lambda
  double* master = nullptr;  // [P + 1]
  double* m = nullptr;       // Adam first moments [P + 1]
  double* v = nullptr;       // Adam second moments [P + 1]
  double* gacc = nullptr;    // accumulated gradient [P + 1]
  double* scal = nullptr;    // [2]: loss partial, spare
  void* dtheta = nullptr;    // one pass's gradient, [P] of the pass's dtype
  int t = 0;                 // Adam steps taken
  double lambda = 1.0;
};

namespace idq {
namespace {

constexpr int kTB = 256;

__global__ __launch_bounds__(kTB) void zero_kernel(double* p, long long n) {
  for (long long i = blockIdx.x * static_cast<long long>(kTB) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * kTB)
    p[i] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(kTB) void accumulate_kernel(double* acc, const T* g, long long n) {
  for (long long i = blockIdx.x * static_cast<long long>(kTB) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * kTB)
    acc[i] += static_cast<double>(g[i]);
}

// Adam (Kingma & Ba) with bias correction, float64:
//   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
//   p <- p - lr (m / bc1) / (sqrt(v / bc2) + eps),  bc_i = 1 - b_i^t.
__global__ __launch_bounds__(kTB) void adam64_kernel(double* p, double* m, double* v,
                                                   const double* g, long long n, double lr,
                                                   double b1, double b2, double eps, double bc1,
                                                   double bc2) {
  for (long long i = blockIdx.x * static_cast<long long>(kTB) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * kTB) {
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (std::sqrt(vi / bc2) + eps);
  }
}

int grid_of(long long n) {
  long long g = (n + kTB - 1) / kTB;
  return static_cast<int>(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

void release(idq_trainer* tr) {
  for (void* q : {static_cast<void*>(tr->master), static_cast<void*>(tr->m),
                  static_cast<void*>(tr->v), static_cast<void*>(tr->gacc),
                  static_cast<void*>(tr->scal), tr->dtheta})
    if (q) (void)hipFree(q);
  tr->master = tr->m = tr->v = tr->gacc = tr->scal = nullptr;
  tr->dtheta = nullptr;
}

int create_impl(idq_trainer** out, idq_ctx* ctx, double lambda0) {
  if (!out || !ctx) return fail(IDQ_E_INVAL, "null argument");
  *out = nullptr;
  if (ctx->L == 0) return fail(IDQ_E_INVAL, "the context has no network to train");
  if (!std::isfinite(lambda0)) return fail(IDQ_E_INVAL, "lambda0 must be finite");
  IDQ_HIP(hipSetDevice(ctx->device));
  auto* tr = new idq_trainer();
  tr->ctx = ctx;
  tr->P = static_cast<long long>(ctx->params.size());
  tr->lambda = lambda0;
  const size_t nb = static_cast<size_t>(tr->P + 1) * sizeof(double);
  auto fail_free = [&](hipError_t e) {
    release(tr);
    delete tr;
    return fail(IDQ_E_NOMEM, std::string("trainer allocation: ") + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipMalloc(&tr->master, nb)) != hipSuccess) return fail_free(e);
  if ((e = hipMalloc(&tr->m, nb)) != hipSuccess) return fail_free(e);
  if ((e = hipMalloc(&tr->v, nb)) != hipSuccess) return fail_free(e);
  if ((e = hipMalloc(&tr->gacc, nb)) != hipSuccess) return fail_free(e);
  if ((e = hipMalloc(&tr->scal, 2 * sizeof(double))) != hipSuccess) return fail_free(e);
  if ((e = hipMalloc(&tr->dtheta, static_cast<size_t>(tr->P) * sizeof(double))) != hipSuccess)
    return fail_free(e);
  std::vector<double> init(ctx->params.begin(), ctx->params.end());
  init.push_back(lambda0);
  IDQ_HIP(hipMemcpy(tr->master, init.data(), nb, hipMemcpyHostToDevice));
  IDQ_HIP(hipMemset(tr->m, 0, nb));
  IDQ_HIP(hipMemset(tr->v, 0, nb));
  *out = tr;
  return IDQ_OK;
}

int epoch_impl(idq_trainer* tr, const void* Y, const void* Xs, const void* X0, int N, int c,
               int h, int w, int dtype, const idq_train_opts* o, double* loss, hipStream_t s) {
  if (!tr || !Y || !Xs || !o) return fail(IDQ_E_INVAL, "null argument");
  if (N <= 0) return fail(IDQ_E_INVAL, "empty dataset");
  if (o->K <= 0) return fail(IDQ_E_INVAL, "K must be positive");
  if (dtype != IDQ_F64 && dtype != IDQ_F32) return fail(IDQ_E_INVAL, "bad dtype");
  if (o->conv_prec != dtype) return fail(IDQ_E_INVAL, "training runs in the tensors' arithmetic");
  if (o->mode != IDQ_BWD_JFB && o->mode != IDQ_BWD_IMPLICIT) return fail(IDQ_E_INVAL, "bad mode");
  idq_ctx* ctx = tr->ctx;
  IDQ_HIP(hipSetDevice(ctx->device));
  Geometry g;
  IDQ_TRY(check_shape(ctx, 1, c, h, w, &g));
  const int batch = o->batch > 0 ? std::min(o->batch, N) : N;
  const size_t es = elem_size(dtype);
  const long long per = g.per;
  const size_t ybytes_per = static_cast<size_t>(per) * es * (ctx->op_kind == IDQ_OP_MRI ? 2 : 1);
  const double d = static_cast<double>(per);
  void *xhat, *vbuf;
  IDQ_TRY(ctx->ws.get(W_TRD, static_cast<size_t>(batch) * per * es, &xhat));
  IDQ_TRY(ctx->ws.get(W_TRV, static_cast<size_t>(batch) * per * es, &vbuf));
  zero_kernel<<<grid_of(tr->P + 1), kTB, 0, s>>>(tr->gacc, tr->P + 1);
  IDQ_HIP(hipGetLastError());
  std::vector<idq_solve_info> info(batch);
  double loss_sum = 0.0, glam = 0.0;
  for (int b0 = 0; b0 < N; b0 += batch) {
    const int nb = std::min(batch, N - b0);
    const char* yb = static_cast<const char*>(Y) + static_cast<size_t>(b0) * ybytes_per;
    const char* xsb = static_cast<const char*>(Xs) + static_cast<size_t>(b0) * per * es;
    const char* x0b = X0 ? static_cast<const char*>(X0) + static_cast<size_t>(b0) * per * es : nullptr;
    // forward: K fixed updates (Alg. 1), x_hat the last iterate or the average
    idq_solve_opts so;
    idq_solve_opts_default(&so);
    so.beta = o->beta;
    so.tau = o->tau;
    so.lambda = tr->lambda;
    so.fixed_iters = o->K;
    so.restart_B = o->restart_B;
    so.conv_prec = dtype;
    so.averaging = o->averaging;
    so.proximal = o->proximal;
    so.poll_every = o->K;
    so.init = IDQ_INIT_Y;
    int rc = solve_internal(ctx, yb, x0b, xhat, nb, c, h, w, dtype, &so, info.data(), s);
    if (rc < 0) return rc;
    for (int i = 0; i < nb; ++i)
      if (info[i].status == IDQ_ST_NONFINITE)
        return fail(IDQ_E_NONFINITE, "a forward pass produced a non-finite iterate");
    // v = dL/dx_hat = 2 (x_hat - x*) / (N d), and the loss partial
    const long long cnt = static_cast<long long>(nb) * per;
    IDQ_TRY(launch_axpbypcz(1.0, xhat, -1.0, xsb, 0.0, nullptr, vbuf, cnt, dtype, s));
    IDQ_TRY(dot_batch(ctx, vbuf, vbuf, cnt, dtype, tr->scal, s));
    double part = 0.0;
    IDQ_HIP(hipMemcpyAsync(&part, tr->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    const double a = 2.0 / (static_cast<double>(N) * d);
    IDQ_TRY(launch_axpbypcz(a, vbuf, 0.0, vbuf, 0.0, nullptr, vbuf, cnt, dtype, s));
    idq_bwd_opts bo;
    std::memset(&bo, 0, sizeof(bo));
    bo.mode = o->mode;
    bo.tau = o->tau;
    bo.lambda = tr->lambda;
    bo.adjoint_max_iter = o->adjoint_max_iter;
    bo.adjoint_tol = o->adjoint_tol;
    bo.proximal = o->proximal;
    idq_bwd_info bi{};
    double dl = 0.0;
    IDQ_TRY(backward_internal(ctx, xhat, yb, vbuf, tr->dtheta, &dl, nb, c, h, w, dtype, &bo, &bi, s));
    if (dtype == IDQ_F64)
      accumulate_kernel<double><<<grid_of(tr->P), kTB, 0, s>>>(
          tr->gacc, static_cast<const double*>(tr->dtheta), tr->P);
    else
      accumulate_kernel<float><<<grid_of(tr->P), kTB, 0, s>>>(
          tr->gacc, static_cast<const float*>(tr->dtheta), tr->P);
    IDQ_HIP(hipGetLastError());
    IDQ_HIP(hipStreamSynchronize(s));
    loss_sum += part / (static_cast<double>(N) * d);
    glam += dl;
  }
  // one Adam step on Theta with the accumulated gradient
  IDQ_HIP(hipMemcpyAsync(tr->gacc + tr->P, &glam, sizeof(double), hipMemcpyHostToDevice, s));
  tr->t += 1;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double bc1 = 1.0 - std::pow(b1, tr->t), bc2 = 1.0 - std::pow(b2, tr->t);
  adam64_kernel<<<grid_of(tr->P), kTB, 0, s>>>(tr->master, tr->m, tr->v, tr->gacc, tr->P,
                                               o->lr_theta, b1, b2, eps, bc1, bc2);
  IDQ_HIP(hipGetLastError());
  if (o->learn_lambda) {
    adam64_kernel<<<1, kTB, 0, s>>>(tr->master + tr->P, tr->m + tr->P, tr->v + tr->P,
                                    tr->gacc + tr->P, 1, o->lr_lambda, b1, b2, eps, bc1, bc2);
    IDQ_HIP(hipGetLastError());
  }
  std::vector<double> host(static_cast<size_t>(tr->P) + 1);
  IDQ_HIP(hipMemcpyAsync(host.data(), tr->master, host.size() * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  IDQ_HIP(hipStreamSynchronize(s));
  ctx->params.assign(host.begin(), host.begin() + tr->P);
  tr->lambda = host[tr->P];
  IDQ_TRY(repack_weights(ctx));
  if (loss) *loss = loss_sum;
  return IDQ_OK;
}

template <class F>
int guard(F&& f) {
  try {
    return f();
  } catch (...) {
    return fail(IDQ_E_INVAL, "unexpected exception in the training loop");
  }
}

}  // namespace
}  // namespace idq

using namespace idq;

extern "C" {

int idq_train_create(idq_trainer** out, idq_ctx* ctx, double lambda0) {
  return guard([&] { return create_impl(out, ctx, lambda0); });
}

int idq_train_destroy(idq_trainer* tr) {
  if (!tr) return IDQ_OK;
  (void)hipSetDevice(tr->ctx->device);
  (void)hipDeviceSynchronize();
  release(tr);
  delete tr;
  return IDQ_OK;
}

int idq_train_epoch(idq_trainer* tr, const void* Y, const void* Xs, const void* X0, int N, int c,
                    int h, int w, int dtype, const idq_train_opts* opts, double* loss,
                    void* stream) {
  return guard([&] {
    return epoch_impl(tr, Y, Xs, X0, N, c, h, w, dtype, opts, loss,
                      static_cast<hipStream_t>(stream));
  });
}

int idq_train_get(idq_trainer* tr, double* theta, double* lambda) {
  return guard([&]() -> int {
    if (!tr) return fail(IDQ_E_INVAL, "null trainer");
    if (theta) std::copy(tr->ctx->params.begin(), tr->ctx->params.end(), theta);
    if (lambda) *lambda = tr->lambda;
    return IDQ_OK;
  });
}

}  // extern "C"
