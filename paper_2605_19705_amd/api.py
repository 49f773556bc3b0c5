"""Python binding of the i-DEQ HIP library with the C ABI's names.

PyTorch supplies device memory and streams only; every step of the method runs
in the library's kernels.  Tensors are CUDA (HIP) tensors, contiguous NCHW,
float64 or float32.

    ctx = IDQ(layers, op_kind="blur", taps=k)      # layers: list of (W, b) arrays
    x, info = ctx.solve(y, beta=0.5, lam=1.0, tau=0.0, power_v0=v0, conv_prec="bf16")
"""
import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

_PREC = {"f64": L.IDQ_F64, "f32": L.IDQ_F32, "bf16": L.IDQ_BF16, "bf16x3": L.IDQ_BF16X3,
         L.IDQ_F64: L.IDQ_F64, L.IDQ_F32: L.IDQ_F32, L.IDQ_BF16: L.IDQ_BF16,
         L.IDQ_BF16X3: L.IDQ_BF16X3}
_OPS = {"identity": L.IDQ_OP_IDENTITY, "blur": L.IDQ_OP_BLUR_CIRC, "tanh_blur": L.IDQ_OP_TANH_BLUR,
        "inpaint": L.IDQ_OP_INPAINT, "mri": L.IDQ_OP_MRI, "rician": L.IDQ_OP_RICIAN}


def _dtype_code(t):
    if t.dtype == torch.float64:
        return L.IDQ_F64
    if t.dtype == torch.float32:
        return L.IDQ_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return C.c_void_p(t.data_ptr())


def _real_dtype(t):
    """Element type of a real tensor, or of a complex tensor's (re, im) parts."""
    if t.dtype == torch.complex128:
        return torch.float64
    if t.dtype == torch.complex64:
        return torch.float32
    return t.dtype


def _kspace(t, like):
    """A complex k-space tensor (MRI data) checked against the image tensor
    ``like``: same (n, c, h, w) and matching element type."""
    if not t.is_complex():
        raise ValueError("MRI data must be a complex tensor")
    if tuple(t.shape) != tuple(like.shape) or _real_dtype(t) != like.dtype:
        raise ValueError("MRI data must match the image shape and precision")
    return t


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _shape4(t):
    if t.dim() != 4:
        raise ValueError("expected an (n, c, h, w) tensor")
    return tuple(int(s) for s in t.shape)


def pack_layers(layers):
    """Flat float64 [W_1, b_1, W_2, b_2, ...] from a list of (W, b)."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float64).ravel(),
                                           np.asarray(b, np.float64).ravel()])
                           for W, b in layers])


@dataclass
class SolveResult:
    iters: np.ndarray
    iters_low: np.ndarray
    iters_mid: np.ndarray
    restarts: np.ndarray
    status: np.ndarray
    rel: np.ndarray
    tau: float
    code: int


class IDQ:
    """One library context: regularizer network + forward operator on a device."""

    def __init__(self, layers=None, act="softplus", op_kind="identity", taps=None, gain=2.0,
                 mask=None, sigma=0.0, device=0):
        lib = L.lib()
        self.layers = [(np.asarray(W, np.float64), np.asarray(b, np.float64))
                       for W, b in (layers or [])]
        nd = L.NetDesc()
        self._params = None
        if self.layers:
            chans = [self.layers[0][0].shape[1]] + [W.shape[0] for W, _ in self.layers]
            nd.n_layers = len(self.layers)
            for i, cch in enumerate(chans):
                nd.channels[i] = cch
            nd.act = L.IDQ_ACT_SOFTPLUS if act == "softplus" else L.IDQ_ACT_IDENTITY
            self._params = np.ascontiguousarray(pack_layers(self.layers))
            nd.params = self._params.ctypes.data_as(C.POINTER(C.c_double))
            self.channels = chans
        else:
            nd.n_layers = 0
            self.channels = []
        od = L.OpDesc()
        od.kind = _OPS[op_kind]
        self._taps = None
        if op_kind in ("blur", "tanh_blur"):
            self._taps = np.ascontiguousarray(np.asarray(taps, np.float64))
            od.kh, od.kw = self._taps.shape
            od.taps = self._taps.ctypes.data_as(C.POINTER(C.c_double))
        od.gain = float(gain)
        self._mask = None
        if op_kind in ("inpaint", "mri"):
            self._mask = np.ascontiguousarray(np.asarray(mask, np.float64))
            od.mh, od.mw = self._mask.shape
            od.mask = self._mask.ctypes.data_as(C.POINTER(C.c_double))
        od.sigma = float(sigma)
        self.op_kind = op_kind
        h = C.c_void_p()
        L.check(lib.idq_create(C.byref(h), C.byref(nd) if self.layers else None, C.byref(od),
                               int(device)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().idq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self):
        return int(L.lib().idq_num_params(self._h))

    def set_params(self, flat):
        flat = np.ascontiguousarray(np.asarray(flat, np.float64))
        L.check(L.lib().idq_set_params(self._h, flat.ctypes.data_as(C.POINTER(C.c_double)),
                                       flat.size))

    # ---- device-time accounting ---------------------------------------------------
    def profile(self, on=True, classes=None, every=1):
        """Time device work per class; ``classes``: names of L.PROF_CLASSES to time
        (all when None); ``every``: time one launch in that many of each class."""
        L.check(L.lib().idq_profile_sample(self._h, int(every)))
        mask = 0
        if on:
            mask = L.IDQ_PROF_ALL if classes is None else sum(1 << L.PROF_CLASSES[c] for c in classes)
        L.check(L.lib().idq_profile_enable(self._h, int(mask)))

    def profile_read(self):
        """{class: (total_ms, launches, pixels)} since the last profile(True)."""
        out = {}
        for name, cls in L.PROF_CLASSES.items():
            ms, n, px = C.c_double(), C.c_longlong(), C.c_double()
            L.check(L.lib().idq_profile_read(self._h, cls, C.byref(ms), C.byref(n), C.byref(px)))
            out[name] = (ms.value, n.value, px.value)
        return out

    # ---- operators -------------------------------------------------------------
    def apply_A(self, x):
        """A(x); complex (same shape) for the MRI operator."""
        if self.op_kind == "mri":
            out = torch.empty(x.shape, device=x.device,
                              dtype=torch.complex128 if x.dtype == torch.float64 else torch.complex64)
        else:
            out = torch.empty_like(x)
        L.check(L.lib().idq_apply_A(self._h, _ptr(x), _ptr(out), *_shape4(x), _dtype_code(x),
                                    _stream()))
        return out

    def apply_AT(self, v, x=None):
        """J_A(x)^T v; v complex for the MRI operator (the result is real)."""
        out = torch.empty(v.shape, device=v.device, dtype=_real_dtype(v))
        L.check(L.lib().idq_apply_AT(self._h, _ptr(x), _ptr(v), _ptr(out), *_shape4(v),
                                     _dtype_code(out), _stream()))
        return out

    def prox_data(self, v, y, tau, out=None):
        """prox_{tau f(., y)}(v) (closed forms; y complex for MRI)."""
        if self.op_kind == "mri":
            _kspace(y, v)
        out = torch.empty_like(v) if out is None else out
        L.check(L.lib().idq_prox_data(self._h, _ptr(v), _ptr(y), float(tau), _ptr(out),
                                      *_shape4(v), _dtype_code(v), _stream()))
        return out

    def grad_data(self, x, y):
        if self.op_kind == "mri":
            _kspace(y, x)
        out = torch.empty_like(x)
        L.check(L.lib().idq_grad_data(self._h, _ptr(x), _ptr(y), _ptr(out), *_shape4(x),
                                      _dtype_code(x), _stream()))
        return out

    def grad_data_noalloc(self, x, y, out=None):
        """grad f(x, y) through the allocation-free entry point; ``out`` may be a
        preallocated tensor (the library itself allocates nothing)."""
        if out is None:
            out = torch.empty_like(x)
        L.check(L.lib().idq_grad_data_noalloc(self._h, _ptr(x), _ptr(y), _ptr(out), *_shape4(x),
                                              _dtype_code(x), _stream()))
        return out

    def grad_reg(self, x, conv_prec=None, with_value=False):
        prec = _PREC[conv_prec] if conv_prec is not None else _dtype_code(x)
        out = torch.empty_like(x)
        gv = np.zeros(x.shape[0]) if with_value else None
        L.check(L.lib().idq_grad_reg(self._h, _ptr(x), _ptr(out),
                                     gv.ctypes.data_as(C.POINTER(C.c_double)) if with_value else None,
                                     *_shape4(x), _dtype_code(x), prec, _stream()))
        return (out, gv) if with_value else out

    def hvp(self, x, v, y=None, lam=1.0, which="reg", conv_prec=None):
        prec = _PREC[conv_prec] if conv_prec is not None else _dtype_code(x)
        out = torch.empty_like(x)
        L.check(L.lib().idq_hvp(self._h, _ptr(x), _ptr(y), _ptr(v), _ptr(out), float(lam),
                                0 if which == "reg" else 1, *_shape4(x), _dtype_code(x), prec,
                                _stream()))
        return out

    def lipschitz(self, x, y, v0, lam=1.0, iters=30, conv_prec=None):
        prec = _PREC[conv_prec] if conv_prec is not None else _dtype_code(x)
        Lv = C.c_double(0.0)
        torch.cuda.current_stream().synchronize()
        L.check(L.lib().idq_lipschitz(self._h, _ptr(x), _ptr(y), _ptr(v0), float(lam), int(iters),
                                      *_shape4(x), _dtype_code(x), prec, C.byref(Lv)))
        return Lv.value

    # ---- solver ------------------------------------------------------------------
    def solve(self, y, x0=None, out=None, beta=0.5, tau=0.0, lam=1.0, tol=1e-4, max_iter=1000,
              fixed_iters=0, restart_B=0.0, grad_at="extrapolated", conv_prec=None,
              switch_tol=2e-3, switch_patience=5, power_iters=30, power_v0=None,
              poll_every=8, init="y", ws=None, ws_prec="bf16", refine_prec="f32",
              history=0, averaging=False, proximal=False, use_graph=True, diverge_ratio=1e6,
              x_prev=None, x_prev_out=None):
        """The i-DEQ forward pass (Alg. 1; Alg. 2 with ``proximal``).  For MRI, y
        is complex k-space data and the iterate is real (x0 default A^T y)."""
        o = L.SolveOpts()
        L.lib().idq_solve_opts_default(C.byref(o))
        o.beta, o.tau, o.lambda_, o.tol = float(beta), float(tau), float(lam), float(tol)
        o.max_iter, o.fixed_iters = int(max_iter), int(fixed_iters)
        o.restart_B = float(restart_B) if restart_B and np.isfinite(restart_B) else 0.0
        o.grad_at = L.IDQ_GRAD_AT_CURRENT if grad_at == "current" else L.IDQ_GRAD_AT_EXTRAPOLATED
        o.conv_prec = (_PREC[conv_prec] if conv_prec is not None
                       else (L.IDQ_F64 if _real_dtype(y) == torch.float64 else L.IDQ_F32))
        o.switch_tol, o.switch_patience = float(switch_tol), int(switch_patience)
        o.power_iters = int(power_iters)
        o.power_v0 = _ptr(power_v0).value if power_v0 is not None else None
        o.poll_every = int(poll_every)
        o.init = {"y": L.IDQ_INIT_Y, "zero": L.IDQ_INIT_ZERO,
                  "warmstart": L.IDQ_INIT_WARMSTART}[init]
        o.ws = ws._h.value if ws is not None else None
        o.ws_prec = _PREC[ws_prec]
        o.refine_prec = _PREC[refine_prec]
        o.averaging = 1 if averaging else 0
        o.proximal = 1 if proximal else 0
        o.use_graph = 1 if use_graph else 0
        o.diverge_ratio = float(diverge_ratio)
        o.x_prev = _ptr(x_prev).value if x_prev is not None else None
        o.x_prev_out = _ptr(x_prev_out).value if x_prev_out is not None else None
        n = y.shape[0]
        rdt = _real_dtype(y)
        if y.is_complex() != (self.op_kind == "mri"):
            raise ValueError("complex k-space data goes with the MRI operator only")
        hist = None
        if history:
            hist = np.full((int(history), n), np.nan)
            o.rel_history = hist.ctypes.data_as(C.POINTER(C.c_double))
            o.history_len = int(history)
        info = (L.SolveInfo * n)()
        x = out if out is not None else torch.empty(y.shape, device=y.device, dtype=rdt)
        code = L.lib().idq_solve(self._h, _ptr(y), _ptr(x0), _ptr(x), *_shape4(y), _dtype_code(x),
                                 C.byref(o), info, _stream())
        L.check(code, allow=(L.IDQ_OK, L.IDQ_W_MAXITER, L.IDQ_E_NONFINITE, L.IDQ_E_DIVERGED))
        res = SolveResult(iters=np.array([i.iters for i in info]),
                          iters_low=np.array([i.iters_low for i in info]),
                          iters_mid=np.array([i.iters_mid for i in info]),
                          restarts=np.array([i.restarts for i in info]),
                          status=np.array([i.status for i in info]),
                          rel=np.array([i.rel for i in info]),
                          tau=float(info[0].tau), code=code)
        res.history = hist
        return x, res

    def backward(self, xbar, y, dl_dx, tau, lam, mode="implicit", adjoint_max_iter=500,
                 adjoint_tol=1e-6, adjoint_beta=0.0, proximal=False):
        o = L.BwdOpts()
        o.proximal = 1 if proximal else 0
        o.mode = L.IDQ_BWD_IMPLICIT if mode == "implicit" else L.IDQ_BWD_JFB
        o.tau, o.lambda_ = float(tau), float(lam)
        o.adjoint_max_iter, o.adjoint_tol = int(adjoint_max_iter), float(adjoint_tol)
        o.adjoint_beta = float(adjoint_beta)
        dtheta = torch.empty(self.num_params, dtype=xbar.dtype, device=xbar.device)
        dlam = C.c_double(0.0)
        info = L.BwdInfo()
        L.check(L.lib().idq_backward(self._h, _ptr(xbar), _ptr(y), _ptr(dl_dx), _ptr(dtheta),
                                     C.byref(dlam), *_shape4(xbar), _dtype_code(xbar), C.byref(o),
                                     C.byref(info), _stream()))
        return dtheta, dlam.value, (info.adjoint_iters, info.adjoint_rel)


class IDQSolve(torch.autograd.Function):
    """x_bar = fixed point of the i-DEQ iteration; gradients by the implicit
    (or JFB) backward of the library.

    Usage: IDQSolve.apply(y, theta, lam, ctx, solve_kwargs, bwd_kwargs) with
    theta the flat network parameters (float64 CPU tensor, loaded into the
    context before the solve) and lam a 0-d tensor.

    The backward differentiates at the returned iterate as if it were the
    fixed point (App. D.1), so the forward raises unless every image either
    met the stopping rule or ran its fixed iteration budget (the paper's
    training runs K iterations): an image that hit max_iter or produced a
    non-finite iterate is an error here.
    """

    @staticmethod
    def forward(fctx, y, theta, lam, ctx, solve_kwargs, bwd_kwargs):
        ctx.set_params(theta.detach().cpu().double().numpy())
        kw = dict(solve_kwargs)
        kw["lam"] = float(lam)
        x, res = ctx.solve(y, **kw)
        bad = [i for i, st in enumerate(res.status) if st not in (L.IDQ_ST_CONVERGED,
                                                                   L.IDQ_ST_FIXED)]
        if bad:
            raise L.IDQError(res.code if res.code != L.IDQ_OK else L.IDQ_W_MAXITER,
                             f"images {bad} did not reach a fixed point "
                             f"(status {[int(res.status[i]) for i in bad]}); "
                             "the implicit backward needs one")
        fctx.save_for_backward(x, y)
        fctx.idq = ctx
        fctx.tau = res.tau
        fctx.lam = float(lam)
        fctx.bwd_kwargs = bwd_kwargs
        fctx.theta_meta = (theta.dtype, theta.device)
        fctx.lam_meta = (lam.dtype, lam.device)
        fctx.res = res
        return x

    @staticmethod
    def backward(fctx, grad_x):
        x, y = fctx.saved_tensors
        dtheta, dlam, _ = fctx.idq.backward(x, y, grad_x.contiguous(), fctx.tau, fctx.lam,
                                            **fctx.bwd_kwargs)
        tdt, tdev = fctx.theta_meta
        ldt, ldev = fctx.lam_meta
        return (None, dtheta.to(device=tdev, dtype=tdt),
                torch.tensor(dlam, dtype=ldt, device=ldev), None, None, None)


class Trainer:
    """The training loop of Alg. 1 / Alg. 2 (``idq_train_*``): Adam on the
    network parameters of ``ctx`` and on lambda, one step per epoch."""

    def __init__(self, ctx, lam0):
        h = C.c_void_p()
        L.check(L.lib().idq_train_create(C.byref(h), ctx._h, float(lam0)))
        self._h = h
        self.ctx = ctx

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().idq_train_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def epoch(self, Y, Xs, X0=None, K=100, beta=0.5, tau=0.1, mode="jfb", restart_B=0.0,
              averaging=False, proximal=False, learn_lambda=True, lr_theta=1e-3,
              lr_lambda=1e-3, adjoint_max_iter=500, adjoint_tol=1e-6, batch=0):
        """One epoch over the N pairs (Y[i], Xs[i]); returns the loss before the step."""
        o = L.TrainOpts()
        o.mode = L.IDQ_BWD_IMPLICIT if mode == "implicit" else L.IDQ_BWD_JFB
        o.K, o.beta, o.tau = int(K), float(beta), float(tau)
        o.restart_B = float(restart_B) if restart_B and np.isfinite(restart_B) else 0.0
        o.averaging, o.proximal = int(bool(averaging)), int(bool(proximal))
        o.conv_prec = _dtype_code(Xs)
        o.learn_lambda = int(bool(learn_lambda))
        o.lr_theta, o.lr_lambda = float(lr_theta), float(lr_lambda)
        o.adjoint_max_iter, o.adjoint_tol = int(adjoint_max_iter), float(adjoint_tol)
        o.batch = int(batch)
        if Y.is_complex():
            _kspace(Y, Xs)
        loss = C.c_double(0.0)
        L.check(L.lib().idq_train_epoch(self._h, _ptr(Y), _ptr(Xs), _ptr(X0), *_shape4(Xs),
                                        _dtype_code(Xs), C.byref(o), C.byref(loss), _stream()))
        return loss.value

    def params(self):
        """(theta as a flat float64 array, lambda)."""
        theta = np.zeros(self.ctx.num_params)
        lam = C.c_double(0.0)
        L.check(L.lib().idq_train_get(self._h, theta.ctypes.data_as(C.POINTER(C.c_double)),
                                      C.byref(lam)))
        return theta, lam.value


class WarmStart:
    """Learned initial iterate x0 = y + W_phi(y) (``idq_ws_*`` of the C ABI).

    ``layers``: the 9 (W, b) pairs of the encoder-decoder, or the flat packed
    parameter vector [W_1, b_1, ..., W_9, b_9].  Images are float32 CUDA
    tensors of shape (n, 3, h, w) with h, w even.
    """

    def __init__(self, layers, device=0):
        lib = L.lib()
        if isinstance(layers, np.ndarray) and layers.ndim == 1:
            flat = np.ascontiguousarray(layers, dtype=np.float64)
        else:
            flat = np.ascontiguousarray(pack_layers(layers))
        n = int(lib.idq_ws_num_params())
        if flat.size != n:
            raise ValueError(f"warm-start network takes {n} parameters, got {flat.size}")
        h = C.c_void_p()
        L.check(lib.idq_ws_create(C.byref(h), flat.ctypes.data_as(C.POINTER(C.c_double)), n,
                                  int(device)))
        self._h = h
        self.device = device
        self.num_params = n

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().idq_ws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(self.num_params, np.float64)
        L.check(L.lib().idq_ws_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(np.asarray(flat, np.float64))
        if flat.size != self.num_params:
            raise ValueError("parameter count mismatch")
        L.check(L.lib().idq_ws_set_params(self._h, flat.ctypes.data_as(C.POINTER(C.c_double))))

    @staticmethod
    def _check(y):
        if y.dtype != torch.float32:
            raise TypeError("warm-start images are float32")
        return _shape4(y)

    def forward(self, y, prec="bf16", out=None):
        n, c, h, w = self._check(y)
        out = torch.empty_like(y) if out is None else out
        L.check(L.lib().idq_ws_forward(self._h, _ptr(y), _ptr(out), n, c, h, w, _PREC[prec],
                                       _stream()))
        return out

    def grad(self, y, target, prec="f32"):
        """(loss, flat float32 gradient tensor) of mean((y + W(y) - target)^2)."""
        n, c, h, w = self._check(y)
        if target.shape != y.shape or target.dtype != torch.float32:
            raise ValueError("target must match y")
        g = torch.empty(self.num_params, dtype=torch.float32, device=y.device)
        loss = C.c_double()
        L.check(L.lib().idq_ws_grad(self._h, _ptr(y), _ptr(target), _ptr(g), n, c, h, w,
                                    _PREC[prec], C.byref(loss), _stream()))
        return loss.value, g

    def train_step(self, y, target, lr, prec="bf16", want_loss=True):
        n, c, h, w = self._check(y)
        if target.shape != y.shape or target.dtype != torch.float32:
            raise ValueError("target must match y")
        loss = C.c_double()
        L.check(L.lib().idq_ws_train_step(self._h, _ptr(y), _ptr(target), n, c, h, w,
                                          _PREC[prec], float(lr),
                                          C.byref(loss) if want_loss else None, _stream()))
        return loss.value if want_loss else None
