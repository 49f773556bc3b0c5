/*
 * idq.h -- C ABI of the i-DEQ inertial fixed-point solver for AMD MI355X (gfx950).
 *
 * The library solves imaging inverse problems y = A(x) + n by minimising
 *     F(x) = f(x, y) + lambda * g(x)                         (paper, eq. inv_prob)
 * with f(x, y) = 1/2 ||A(x) - y||^2 and the learned gradient-step potential
 *     g(x) = 1/2 ||x - N_theta(x)||^2                        (paper, Sec. 2.2, eq. GS)
 * where N_theta is a stack of zero-padded 3x3 conv layers with SoftPlus
 * activations.  The solver is the i-DEQ iteration (eq. ideq, Alg. 1):
 *     z^k     = x^k + beta (x^k - x^{k-1})                    (eq. Momentum, beta = 1 - alpha)
 *     x^{k+1} = z^k - tau (grad f(z^k, y) + lambda grad g(z^k))
 * with the adaptive restart of eq. restart and the per-image stopping rule
 * ||x^{k+1} - x^k|| / ||x^k|| < tol of App. D.1.3.
 *
 * Conventions shared by every call
 *   - Image tensors are dense, contiguous NCHW arrays (n images, c channels,
 *     h rows, w columns) in DEVICE memory owned by the caller; element type is
 *     given by `dtype` (IDQ_F64 = double, IDQ_F32 = float).  The library never
 *     frees or keeps caller pointers beyond the call.
 *   - If the network's input channel count is 1 and c > 1, N_theta is applied
 *     to every channel as a separate grey image; otherwise c must equal it.
 *   - Host arrays are marked "host"; everything else is a device pointer.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All calls are
 *     asynchronous on `stream` unless stated otherwise.
 *   - A context is not thread safe; use one per host thread.
 *   - Every call returns IDQ_OK (0), a positive warning or a negative error;
 *     idq_last_error() returns a thread-local message for the last failure.
 *     No C++ exception crosses this interface.
 */
#ifndef IDQ_H
#define IDQ_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define IDQ_OK              0
#define IDQ_W_MAXITER       1   /* some image hit max_iter; results written   */
#define IDQ_E_INVAL        -1   /* null pointer, bad shape, dtype or option    */
#define IDQ_E_NOMEM        -2   /* device allocation failed                    */
#define IDQ_E_HIP          -3   /* HIP runtime error (message has the reason)  */
#define IDQ_E_NONFINITE    -4   /* a non-finite iterate was produced           */
#define IDQ_E_UNSUPPORTED  -5   /* option combination not implemented          */
#define IDQ_E_DIVERGED     -6   /* an image's iterate passed diverge_ratio x ||x^0|| */

/* ---- element / arithmetic types ---------------------------------------- */
#define IDQ_F64   0
#define IDQ_F32   1
#define IDQ_BF16  2   /* conv arithmetic only: bf16 operands, fp32 accumulate */
#define IDQ_BF16X3 3  /* conv arithmetic only: each float32 operand split into bf16
                         hi + lo parts, three bf16 products per term (hi*hi + lo*hi +
                         hi*lo) accumulated in fp32 -- products good to ~2^-16
                         relative; float32 activations.  Layers without a split
                         kernel (image-facing ones) run in IDQ_F32. */

/* ---- activations, operators, options ------------------------------------ */
#define IDQ_ACT_SOFTPLUS   0
#define IDQ_ACT_IDENTITY   1

#define IDQ_OP_IDENTITY    0   /* A(x) = x                                     */
#define IDQ_OP_BLUR_CIRC   1   /* A x = k (*) x, circular cross-correlation     */
#define IDQ_OP_TANH_BLUR   2   /* A(x) = tanh(gain * (k (*) x)) / tanh(gain)    */
#define IDQ_OP_INPAINT     3   /* A x = M . x, M an h x w 0/1 pixel mask applied
                                  to every channel (App. D.3.2)                  */
#define IDQ_OP_MRI         4   /* A x = M . F x, F the unitary 2-D DFT of each
                                  plane, M an h x w 0/1 k-space mask (App. D.3.1);
                                  x is real (the phase is fixed to zero), y and
                                  A(x) are complex: n*c*h*w (re, im) pairs of
                                  dtype.  h and w: powers of two in [4, 1024]    */
#define IDQ_OP_RICIAN      5   /* Rician likelihood instead of a Gaussian one
                                  (App. D.3.3): A = identity and
                                  f(x, y) = sum x^2/(2 s^2) - log I_0(x y / s^2) */

#define IDQ_GRAD_AT_EXTRAPOLATED 0   /* gradient at z^k (Alg. 1)             */
#define IDQ_GRAD_AT_CURRENT      1   /* gradient at x^k (heavy-ball form)    */

#define IDQ_INIT_Y          0
#define IDQ_INIT_ZERO       1
#define IDQ_INIT_WARMSTART  2

#define IDQ_MAX_LAYERS 8

/* per-image status in idq_solve_info.status */
#define IDQ_ST_CONVERGED   0
#define IDQ_ST_MAXITER     1
#define IDQ_ST_FIXED       2
#define IDQ_ST_NONFINITE  -4
#define IDQ_ST_DIVERGED   -6   /* iterate norm above diverge_ratio: stopped     */

typedef struct idq_ctx idq_ctx;
typedef struct idq_ws idq_ws;

/* Regularizer network N_theta (paper, Sec. 2.2 eq. GS; SoftPlus as in Sec. 3.3).
 * channels[0..n_layers]: channels[0] == channels[n_layers] (N maps images to images).
 * params (host, float64): packed [W_1, b_1, W_2, b_2, ...] with W_l in C order
 * (c_out, c_in, 3, 3) and b_l (c_out).  The activation follows every layer but
 * the last.  Copied at create time. */
typedef struct {
    int n_layers;                      /* 1..IDQ_MAX_LAYERS                     */
    int channels[IDQ_MAX_LAYERS + 1];
    int act;                           /* IDQ_ACT_*                             */
    const double* params;              /* host                                  */
} idq_net_desc;

/* Forward operator A (paper, eq. inv_prob; the blur operators are the
 * deblurring and nonlinear workloads).  taps (host, float64): kh x kw row-major,
 * kh and kw odd, centred; the correlation is
 *   (B x)[i,j] = sum_{a,b} k[a,b] x[(i+a-(kh-1)/2) mod h, (j+b-(kw-1)/2) mod w].
 * For a Gaussian noise model f(x, y) = 1/2 ||A(x) - y||^2, so
 * grad f = J_A^T (A(x) - y); for real x and complex MRI data the inner product
 * is Re<u, v> and grad f = Re(F^H M (M F x - y)) (App. D.3.1-2).
 * mask (host, float64, mh x mw of 0 or 1, copied at create time): the pixel
 * mask of IDQ_OP_INPAINT, or the k-space mask of IDQ_OP_MRI in the DFT's own
 * index order (frequency 0 at index 0); images must then be mh x mw. */
typedef struct {
    int kind;                          /* IDQ_OP_*                              */
    int kh, kw;                        /* taps size (blurs only)                */
    const double* taps;                /* host, copied at create time           */
    double gain;                       /* tanh-blur gamma (e.g. 2.0)            */
    const double* mask;                /* host; INPAINT and MRI only            */
    int mh, mw;                        /* mask rows and columns                 */
    double sigma;                      /* RICIAN: noise level sigma_y > 0       */
} idq_op_desc;

/* Options of idq_solve.  Fill with idq_solve_opts_default() first. */
typedef struct {
    double beta;            /* inertia beta = 1 - alpha (eq. Momentum)          */
    double tau;             /* step size; 0 => 0.9 / L by power iteration        */
    double lambda;          /* regularisation weight                             */
    double tol;             /* stopping tolerance on the relative residual       */
    int    max_iter;        /* per-image iteration cap                           */
    int    fixed_iters;     /* > 0: exactly this many updates, tol ignored       */
    double restart_B;       /* restart threshold B (eq. restart); <= 0 => off    */
    int    grad_at;         /* IDQ_GRAD_AT_*                                     */
    int    conv_prec;       /* IDQ_F64 (dtype F64 only) | IDQ_F32 | IDQ_BF16 |
                               IDQ_BF16X3                                         */
    double switch_tol;      /* BF16 phase ends when rel < switch_tol (default
                               2e-3) ...                                          */
    int    switch_patience; /* ... or after this many BF16 steps with no new best
                               (default 5)                                        */
    int    power_iters;     /* power iterations when tau == 0                    */
    const void* power_v0;   /* device, shape of y: power-iteration start vector  */
    int    poll_every;      /* iterations enqueued between host polls of the
                               per-image phases (default 8; <= 0 => 8).  Passes of a phase
                               no image can be in are skipped; an image that
                               reaches the float32 phase before its passes are
                               launched waits (no update, no count) until they
                               are.  The iterates do not depend on this value,
                               only the launch count and the sync cost do.     */
    int    init;            /* IDQ_INIT_* used when x0 == NULL                    */
    idq_ws* ws;             /* warm-start network for IDQ_INIT_WARMSTART          */
    int    ws_prec;         /* IDQ_F32 | IDQ_BF16 for the warm-start inference    */
    int    refine_prec;     /* with conv_prec == IDQ_BF16: IDQ_F32 (default): the
                               BF16 phase hands over to float32; IDQ_BF16X3: to a
                               split-bf16 phase that runs until rel < tol (or
                               stagnates), then float32 updates until rel < tol.
                               An image stops only on a float32 update.          */
    double* rel_history;    /* host, nullable: n * history_len doubles; entry
                               [k * n + i] = relative residual of image i after
                               update k+1 (NaN once the image has stopped)        */
    int    history_len;     /* rows of rel_history (updates recorded)             */
    int    averaging;       /* 1: return the averaged iterate of Alg. 1's last
                               step instead of x^K:
                                 K_0 = argmin_{floor(K/2) < k < K-1} ||x^{k+1}-x^k||
                                 (the first such k on ties),
                                 x_hat = (K_0 + 1)^{-1} sum_{k=0..K_0} z^k,
                               with K = fixed_iters; x^0 if the window is empty
                               (K < 4).  Needs fixed_iters > 0, restart off and
                               a single arithmetic (conv_prec != IDQ_BF16), else
                               IDQ_E_UNSUPPORTED.  Remark 1 of the paper notes
                               that the step may be omitted; 0 (default) omits it. */
    int    proximal;        /* 1: i-DEQ-P (App. B, Alg. 2): the update is
                                 x^{k+1} = prox_{tau f(., y)}(z^k - tau lambda grad g(z^k))
                               with the closed-form prox of idq_prox_data; needs
                               grad_at = EXTRAPOLATED and an operator with a
                               closed form (identity, blur, inpainting, MRI),
                               else IDQ_E_UNSUPPORTED.  0 (default): Alg. 1.     */
    double diverge_ratio;   /* an image whose iterate norm ||x^k|| exceeds this
                               times ||x^0|| (||x^1|| when x^0 = 0) stops with
                               IDQ_ST_DIVERGED (default 1e6; <= 0: off).  With tau
                               too large for the curvature the iterates grow
                               geometrically while the relative step stays
                               bounded, so the norm is what is tested.          */
    const void* x_prev;     /* device, nullable: x^{-1} of a resumed iteration; the
                               first step then extrapolates with beta (restart
                               counters start from zero).  NULL: x^{-1} = x^0.     */
    void*  x_prev_out;      /* device, nullable: receives each image's iterate
                               before x_out (x_out itself where the last update
                               restarted the inertia), so that (x_out, x_prev_out)
                               as (x0, x_prev) continues the iteration exactly.   */
    int    use_graph;       /* 1 (default): a solve of fixed_iters >= 3 updates in
                               one conv arithmetic, without averaging or device-time
                               accounting, replays its steps from a HIP graph on
                               a stream of the context (ordered after and before
                               `stream` by events); results are identical.
                               0: every kernel is launched one by one.           */
} idq_solve_opts;

/* Per-image results of idq_solve (host array of n entries). */
typedef struct {
    int    iters;           /* updates performed                                  */
    int    iters_low;       /* of which in the BF16 phase                          */
    int    restarts;        /* restarts fired                                      */
    int    status;          /* IDQ_ST_*                                            */
    double rel;             /* last relative residual ||x^{k+1}-x^k|| / ||x^k||    */
    double tau;             /* step size used                                      */
    int    iters_mid;       /* of which in the split-bf16 phase                    */
} idq_solve_info;

#define IDQ_BWD_JFB       0   /* Jacobian-free backprop: adjoint u = v           */
#define IDQ_BWD_IMPLICIT  1   /* adjoint fixed point u = (I - tau H) u + v        */

typedef struct {
    int    mode;              /* IDQ_BWD_*                                       */
    double tau, lambda;       /* the forward pass's step size and weight          */
    int    adjoint_max_iter;
    double adjoint_tol;       /* on ||u_{j+1} - u_j|| / ||u_j|| (batch norms),
                                 tested every 8 iterations and at the last one    */
    double adjoint_beta;      /* inertia applied to the adjoint iteration          */
    int    proximal;          /* 1: the fixed point is i-DEQ-P's (App. B, Alg. 2):
                                 the map is P(z - tau lambda grad g(z)) with the
                                 prox's Jacobian J_P = (I + tau A^T A)^{-1}, so
                                 JFB uses J_P v and IMPLICIT solves
                                 u = (I - tau lambda H_g) J_P u + v and uses J_P u */
} idq_bwd_opts;

typedef struct {
    int    adjoint_iters;
    double adjoint_rel;
} idq_bwd_info;

/* ---- library ------------------------------------------------------------- */
const char* idq_last_error(void);          /* thread-local message, never NULL  */
int idq_version(void);                     /* 10000*major + 100*minor + patch   */
void idq_solve_opts_default(idq_solve_opts* o);  /* host; beta .5, lambda 1, tol
                                              1e-4, max_iter 1000, F32, ...       */

/* Create a context on HIP device `device` for the problem y = A(x) + n solved
 * as argmin f + lambda g (eq. inv_prob, eq. GS): copies the network and the
 * operator, packs the weights for every conv arithmetic.  net may be NULL
 * (g = 0).  Synchronous. */
int idq_create(idq_ctx** out, const idq_net_desc* net, const idq_op_desc* op, int device);
/* Destroy a context and free its device memory.  Synchronous. */
int idq_destroy(idq_ctx* ctx);
/* Replace the network parameters (host float64, packed as in idq_net_desc);
 * `count` must equal the packed size.  Synchronous. */
int idq_set_params(idq_ctx* ctx, const double* params, long long count);
/* Number of packed network parameters. */
long long idq_num_params(const idq_ctx* ctx);

/* Ax = A(x) (eq. inv_prob).  x, Ax: n*c*h*w of dtype (MRI: Ax complex, see
 * IDQ_OP_MRI).  The Rician model has no operator (IDQ_E_UNSUPPORTED). */
int idq_apply_A(idq_ctx* ctx, const void* x, void* Ax, int n, int c, int h, int w,
                int dtype, void* stream);
/* out = J_A(x)^T v, the adjoint (transposed Jacobian) of A at x (eq. inv_prob,
 * grad f = J_A^T (A x - y)); x may be NULL for the linear operators.  MRI: v
 * complex, out = Re(F^H (M v)) real. */
int idq_apply_AT(idq_ctx* ctx, const void* x, const void* v, void* out,
                 int n, int c, int h, int w, int dtype, void* stream);
/* grad = grad_x f(x, y) = J_A(x)^T (A(x) - y); Rician:
 * x / s^2 - (y / s^2) I_1(x y / s^2) / I_0(x y / s^2) (App. D.3.3).  MRI: y complex. */
int idq_grad_data(idq_ctx* ctx, const void* x, const void* y, void* grad,
                  int n, int c, int h, int w, int dtype, void* stream);
/* grad = grad g(x) = r - J_N(x)^T r, r = x - N(x) (derivative of eq. GS).
 * g_val (host, nullable): n per-image values of g; when given the call is
 * synchronous.  conv_prec: IDQ_F64 (dtype F64) | IDQ_F32 | IDQ_BF16. */
int idq_grad_reg(idq_ctx* ctx, const void* x, void* grad, double* g_val,
                 int n, int c, int h, int w, int dtype, int conv_prec, void* stream);
/* out = H v with H = Hessian of g at x (which = 0) or of F = f + lambda g at
 * (x, y) (which = 1; eq. inv_prob and the second derivative of eq. GS, the
 * operator of the implicit backward, App. D.1); y may be NULL for which = 0. */
int idq_hvp(idq_ctx* ctx, const void* x, const void* y, const void* v, void* out,
            double lambda, int which, int n, int c, int h, int w, int dtype,
            int conv_prec, void* stream);
/* The step size of the i-DEQ iteration is tau = 0.9 / L (workload configuration;
 * the paper states L_f = 1 for its linear operators, App. D.3.1-2).
 * L = largest-magnitude eigenvalue of the batch Hessian of F at (x, y) by
 * `iters` steps of v <- Hv/||Hv|| from v0 (device, same shape), L = <v, Hv>.
 * Norms and dots in float64.  L (host) is written; synchronous. */
int idq_lipschitz(idq_ctx* ctx, const void* x, const void* y, const void* v0,
                  double lambda, int iters, int n, int c, int h, int w, int dtype,
                  int conv_prec, double* L);
/* The i-DEQ forward pass (Alg. 1) on a batch of n independent images.
 * y: measurements; x0: initial iterate or NULL (then opts->init); x_out: the
 * returned iterate of every image (the first iterate meeting the stopping
 * rule, or the last one).  info: host array of n entries.  Synchronous: it
 * returns after every image stopped.  Returns IDQ_OK, IDQ_W_MAXITER if some
 * image hit max_iter, or IDQ_E_NONFINITE if some image produced a non-finite
 * iterate (its status says which; other images are still valid). */
int idq_solve(idq_ctx* ctx, const void* y, const void* x0, void* x_out,
              int n, int c, int h, int w, int dtype, const idq_solve_opts* opts,
              idq_solve_info* info, void* stream);
/* out = prox_{tau f(., y)}(v) = argmin_x f(x, y) + ||x - v||^2 / (2 tau) (App. B,
 * eq. red_prox), for the operators with a closed form: identity, inpainting
 * ((v + tau M y) / (1 + tau M), App. D.3.2), circular blur and MRI (the
 * normal equations (I + tau A^T A) x = v + tau A^T y solved in the Fourier
 * domain; for the real-valued MRI problem A^T A = F^H M_s F with
 * M_s(k) = (M(k) + M(-k)) / 2).  Blur and MRI need power-of-two h, w in
 * [4, 1024].  Tanh-blur and Rician: IDQ_E_UNSUPPORTED. */
int idq_prox_data(idq_ctx* ctx, const void* v, const void* y, double tau, void* out,
                  int n, int c, int h, int w, int dtype, void* stream);
/* Gradient of a loss through the fixed point xbar (paper, App. D.1):
 * dl_dx = dloss/dxbar (device, image shaped).  Writes dtheta (device, dtype,
 * packed like the network parameters) and *dlambda (host).  IMPLICIT solves
 * u = (I - tau H_F(xbar)) u + v by fixed-point iteration; JFB uses u = v.
 * dtheta = -tau lambda d/dtheta <u, grad g(xbar)>, dlambda = -tau <grad g, u>.
 * Synchronous. */
int idq_backward(idq_ctx* ctx, const void* xbar, const void* y, const void* dl_dx,
                 void* dtheta, double* dlambda, int n, int c, int h, int w, int dtype,
                 const idq_bwd_opts* opts, idq_bwd_info* info, void* stream);

/* ---- training loop (Alg. 1, Alg. 2) ----------------------------------------
 * One epoch of Alg. 1 over a dataset of N pairs (y_i, x*_i): the gradient of
 * the epoch loss L = (1/N) sum_i mean_pixels (x_hat_i - x*_i)^2 is accumulated
 * over the pairs, each x_hat_i the output of K fixed updates of the i-DEQ
 * iteration (with restart and the averaging step as configured), then one Adam
 * step (betas 0.9 / 0.999, eps 1e-8, bias-corrected) updates Theta = {theta,
 * lambda}.  tau and beta stay fixed: their derivatives vanish at an exact fixed
 * point (App. D.1.2).  The trainer keeps float64 master parameters and Adam
 * moments on the device and loads the updated theta into its context after
 * every step. */
typedef struct idq_trainer idq_trainer;
typedef struct {
    int    mode;              /* IDQ_BWD_JFB | IDQ_BWD_IMPLICIT                    */
    int    K;                 /* forward updates per pair (Alg. 1's budget)        */
    double beta, tau;         /* inertia and step size of the forward pass         */
    double restart_B;         /* <= 0: no restart                                   */
    int    averaging;         /* 1: the averaging step gives x_hat                  */
    int    proximal;          /* 1: i-DEQ-P (Alg. 2)                                */
    int    conv_prec;         /* IDQ_F64 (dtype F64) | IDQ_F32                      */
    int    learn_lambda;      /* 0: lambda stays fixed                              */
    double lr_theta, lr_lambda;
    int    adjoint_max_iter;
    double adjoint_tol;
    int    batch;             /* pairs per pass over the GPU (<= N; 0: all)        */
} idq_train_opts;
/* ctx: the problem (operator, network whose parameters are trained); lambda0:
 * the initial weight.  The trainer uses ctx for every pass; it must outlive
 * the trainer.  Synchronous. */
int idq_train_create(idq_trainer** out, idq_ctx* ctx, double lambda0);
int idq_train_destroy(idq_trainer* tr);
/* One epoch.  Y: N measurements (device, dtype; MRI: complex), Xs: N targets,
 * X0: N initial iterates or NULL (then y; MRI: A^T y).  loss (host): L before
 * the step.  Synchronous. */
int idq_train_epoch(idq_trainer* tr, const void* Y, const void* Xs, const void* X0, int N, int c,
                    int h, int w, int dtype, const idq_train_opts* opts, double* loss,
                    void* stream);
/* Current parameters: theta (host, packed like idq_net_desc.params) and lambda. */
int idq_train_get(idq_trainer* tr, double* theta, double* lambda);

/* ---- allocation-free variant ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * idq_grad_data_noalloc computes exactly what idq_grad_data computes, with the
 * same kernels, but stages its intermediate image (A(x) - y for the blur, the
 * tanh-weighted residual for the tanh-blur) in a fixed device array of
 * IDQ_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  It calls no allocating routine.  The intermediate
 * image needs n*c*h*w elements of dtype; larger inputs return IDQ_E_INVAL
 * with a message.  The identity, inpainting and Rician terms need no scratch
 * (their gradients are pixelwise); the MRI operator is not served
 * (IDQ_E_UNSUPPORTED).
 * Every call on one GPU shares that GPU's array, from every context: calls
 * whose executions overlap on one GPU (concurrent streams, several host
 * threads) race on it and must be serialised by the caller. */
#define IDQ_NOALLOC_SCRATCH_BYTES (32LL << 20)
int idq_grad_data_noalloc(idq_ctx* ctx, const void* x, const void* y, void* grad,
                          int n, int c, int h, int w, int dtype, void* stream);

/* ---- device-time accounting ------------------------------------------------
 * When enabled, the library brackets its kernel launches with HIP events on
 * the launch stream and counts the output pixels each conv pass computed
 * (images frozen by the stopping rule are skipped, so only done work counts).
 * Classes: */
#define IDQ_PROF_CONV64_BF16   0   /* 64->64-channel conv passes, bf16 MFMA     */
#define IDQ_PROF_CONV64_F32    1   /* 64->64-channel conv passes, fp32 MFMA     */
#define IDQ_PROF_CONV_OTHER    2   /* every other conv pass                      */
#define IDQ_PROF_STENCIL       3   /* blur stencils of grad f                    */
#define IDQ_PROF_UPDATE        4   /* extrapolation, update, finalize            */
#define IDQ_PROF_WARMSTART     5   /* warm-start network inference               */
#define IDQ_PROF_CONV64_BF16X3 6   /* 64->64-channel conv passes, split-bf16 MFMA */
/* Accounting of device time per class: on == 0 disables it; otherwise `on` is
 * the bit mask of the classes to time (1 << IDQ_PROF_*; IDQ_PROF_ALL for all).
 * Each timed launch costs its events (conv classes: stamped by the dispatch
 * itself; the others: recorded around the launch).  Resets all counters.
 * Synchronous. */
#define IDQ_PROF_ALL 0x7fffffff
int idq_profile_enable(idq_ctx* ctx, int on);
/* Time only one launch in `every` (>= 1; default 1) of each timed class: the
 * first launch after the enable and then every `every`-th, counted per class.
 * The read-out then covers the sampled launches only (an average per launch
 * stays unbiased when `every` is coprime with the launch pattern), and the
 * event packets, which hold the queue a few microseconds each, cost 1/`every`
 * as much.  Restarts the per-class launch count; kept across enables.
 * IDQ_E_INVAL for every < 1. */
int idq_profile_sample(idq_ctx* ctx, int every);
/* Totals since the last enable: summed device time (ms), number of launches
 * and output pixels computed (conv classes; 0 otherwise).  Synchronous. */
int idq_profile_read(idq_ctx* ctx, int cls, double* total_ms, long long* launches,
                     double* pixels);

/* ---- learned warm start x0 = y + W_phi(y) ---------------------------------
 * 2-level encoder-decoder on 3-channel images (h, w even):
 *   3->32->32 | avgpool 2x2 | 32->64->64->64->64 | nearest upsample |
 *   concat(upsampled 64, skip 32) | 96->32->32->3, SoftPlus after all but the last.
 * params (host, float64): the 9 convs packed like idq_net_desc.params. */
int idq_ws_create(idq_ws** out, const double* params, long long count, int device);
int idq_ws_destroy(idq_ws* ws);
long long idq_ws_num_params(void);
int idq_ws_get_params(idq_ws* ws, double* params);          /* host out; sync  */
int idq_ws_set_params(idq_ws* ws, const double* params);    /* host in; sync   */
/* x0 = y + W_phi(y); y, x0: float32 NCHW with c == 3.  prec: F32 | BF16. */
int idq_ws_forward(idq_ws* ws, const void* y, void* x0, int n, int c, int h, int w,
                   int prec, void* stream);
/* One Adam step (lr, betas 0.9/0.999, eps 1e-8) on the mean squared error
 * between y + W_phi(y) and target (float32 NCHW).  Master weights float32;
 * prec selects the conv arithmetic.  loss (host, nullable) receives the loss
 * before the step; synchronous when loss != NULL. */
int idq_ws_train_step(idq_ws* ws, const void* y, const void* target, int n, int c,
                      int h, int w, int prec, double lr, double* loss, void* stream);
/* Gradient of the same loss w.r.t. the parameters without updating them:
 * grad (device, float32, packed like params).  loss as above. */
int idq_ws_grad(idq_ws* ws, const void* y, const void* target, void* grad, int n,
                int c, int h, int w, int prec, double* loss, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* IDQ_H */
