"""ctypes declarations of libidq.so (the C ABI in include/idq.h).

Argument marshalling only: every computation happens inside the HIP library.
Loading fails loudly if the library has not been built (there is no fallback).
"""
import ctypes as C
import os

import torch  # noqa: F401  (load torch's HIP runtime first so the library shares it)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libidq.so")

IDQ_OK, IDQ_W_MAXITER = 0, 1
IDQ_E_INVAL, IDQ_E_NOMEM, IDQ_E_HIP, IDQ_E_NONFINITE, IDQ_E_UNSUPPORTED = -1, -2, -3, -4, -5
IDQ_E_DIVERGED = -6
IDQ_F64, IDQ_F32, IDQ_BF16, IDQ_BF16X3 = 0, 1, 2, 3
IDQ_ACT_SOFTPLUS, IDQ_ACT_IDENTITY = 0, 1
IDQ_OP_IDENTITY, IDQ_OP_BLUR_CIRC, IDQ_OP_TANH_BLUR = 0, 1, 2
IDQ_OP_INPAINT, IDQ_OP_MRI, IDQ_OP_RICIAN = 3, 4, 5
IDQ_GRAD_AT_EXTRAPOLATED, IDQ_GRAD_AT_CURRENT = 0, 1
IDQ_INIT_Y, IDQ_INIT_ZERO, IDQ_INIT_WARMSTART = 0, 1, 2
IDQ_MAX_LAYERS = 8
IDQ_ST_CONVERGED, IDQ_ST_MAXITER, IDQ_ST_FIXED, IDQ_ST_NONFINITE = 0, 1, 2, -4
IDQ_ST_DIVERGED = -6
IDQ_BWD_JFB, IDQ_BWD_IMPLICIT = 0, 1
IDQ_PROF_ALL = 0x7fffffff
IDQ_NOALLOC_SCRATCH_BYTES = 32 << 20
PROF_CLASSES = {"conv64_bf16": 0, "conv64_f32": 1, "conv_other": 2, "stencil": 3, "update": 4,
                "warmstart": 5, "conv64_bf16x3": 6}

EXPORTED = [
    "idq_last_error", "idq_version", "idq_solve_opts_default", "idq_create", "idq_destroy",
    "idq_set_params", "idq_num_params", "idq_apply_A", "idq_apply_AT", "idq_grad_data",
    "idq_grad_reg", "idq_hvp", "idq_lipschitz", "idq_solve", "idq_backward", "idq_prox_data",
    "idq_train_create", "idq_train_destroy", "idq_train_epoch", "idq_train_get",
    "idq_profile_enable", "idq_profile_sample", "idq_profile_read", "idq_grad_data_noalloc",
    "idq_ws_create", "idq_ws_destroy", "idq_ws_num_params", "idq_ws_get_params",
    "idq_ws_set_params", "idq_ws_forward", "idq_ws_train_step", "idq_ws_grad",
]


class NetDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("channels", C.c_int * (IDQ_MAX_LAYERS + 1)),
                ("act", C.c_int), ("params", C.POINTER(C.c_double))]


class OpDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("kh", C.c_int), ("kw", C.c_int),
                ("taps", C.POINTER(C.c_double)), ("gain", C.c_double),
                ("mask", C.POINTER(C.c_double)), ("mh", C.c_int), ("mw", C.c_int),
                ("sigma", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("beta", C.c_double), ("tau", C.c_double), ("lambda_", C.c_double),
                ("tol", C.c_double), ("max_iter", C.c_int), ("fixed_iters", C.c_int),
                ("restart_B", C.c_double), ("grad_at", C.c_int), ("conv_prec", C.c_int),
                ("switch_tol", C.c_double), ("switch_patience", C.c_int),
                ("power_iters", C.c_int), ("power_v0", C.c_void_p), ("poll_every", C.c_int),
                ("init", C.c_int), ("ws", C.c_void_p), ("ws_prec", C.c_int),
                ("refine_prec", C.c_int), ("rel_history", C.POINTER(C.c_double)),
                ("history_len", C.c_int), ("averaging", C.c_int), ("proximal", C.c_int),
                ("diverge_ratio", C.c_double), ("x_prev", C.c_void_p), ("x_prev_out", C.c_void_p),
                ("use_graph", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("iters_low", C.c_int), ("restarts", C.c_int),
                ("status", C.c_int), ("rel", C.c_double), ("tau", C.c_double),
                ("iters_mid", C.c_int)]


class BwdOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("tau", C.c_double), ("lambda_", C.c_double),
                ("adjoint_max_iter", C.c_int), ("adjoint_tol", C.c_double),
                ("adjoint_beta", C.c_double), ("proximal", C.c_int)]


class TrainOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("K", C.c_int), ("beta", C.c_double), ("tau", C.c_double),
                ("restart_B", C.c_double), ("averaging", C.c_int), ("proximal", C.c_int),
                ("conv_prec", C.c_int), ("learn_lambda", C.c_int), ("lr_theta", C.c_double),
                ("lr_lambda", C.c_double), ("adjoint_max_iter", C.c_int),
                ("adjoint_tol", C.c_double), ("batch", C.c_int)]


class BwdInfo(C.Structure):
    _fields_ = [("adjoint_iters", C.c_int), ("adjoint_rel", C.c_double)]


_lib = None

vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
_SIGS = {
    "idq_last_error": ([], C.c_char_p),
    "idq_version": ([], C.c_int),
    "idq_solve_opts_default": ([C.POINTER(SolveOpts)], None),
    "idq_create": ([C.POINTER(vp), C.POINTER(NetDesc), C.POINTER(OpDesc), ip], ip),
    "idq_destroy": ([vp], ip),
    "idq_set_params": ([vp, dp, C.c_longlong], ip),
    "idq_num_params": ([vp], C.c_longlong),
    "idq_apply_A": ([vp, vp, vp, ip, ip, ip, ip, ip, vp], ip),
    "idq_apply_AT": ([vp, vp, vp, vp, ip, ip, ip, ip, ip, vp], ip),
    "idq_grad_data": ([vp, vp, vp, vp, ip, ip, ip, ip, ip, vp], ip),
    "idq_grad_reg": ([vp, vp, vp, dp, ip, ip, ip, ip, ip, ip, vp], ip),
    "idq_hvp": ([vp, vp, vp, vp, vp, C.c_double, ip, ip, ip, ip, ip, ip, ip, vp], ip),
    "idq_lipschitz": ([vp, vp, vp, vp, C.c_double, ip, ip, ip, ip, ip, ip, ip, dp], ip),
    "idq_solve": ([vp, vp, vp, vp, ip, ip, ip, ip, ip, C.POINTER(SolveOpts),
                   C.POINTER(SolveInfo), vp], ip),
    "idq_backward": ([vp, vp, vp, vp, vp, dp, ip, ip, ip, ip, ip, C.POINTER(BwdOpts),
                      C.POINTER(BwdInfo), vp], ip),
    "idq_grad_data_noalloc": ([vp, vp, vp, vp, ip, ip, ip, ip, ip, vp], ip),
    "idq_prox_data": ([vp, vp, vp, C.c_double, vp, ip, ip, ip, ip, ip, vp], ip),
    "idq_train_create": ([C.POINTER(vp), vp, C.c_double], ip),
    "idq_train_destroy": ([vp], ip),
    "idq_train_epoch": ([vp, vp, vp, vp, ip, ip, ip, ip, ip, C.POINTER(TrainOpts), dp, vp], ip),
    "idq_train_get": ([vp, dp, dp], ip),
    "idq_profile_enable": ([vp, ip], ip),
    "idq_profile_sample": ([vp, ip], ip),
    "idq_profile_read": ([vp, ip, dp, C.POINTER(C.c_longlong), dp], ip),
    "idq_ws_create": ([C.POINTER(vp), dp, C.c_longlong, ip], ip),
    "idq_ws_destroy": ([vp], ip),
    "idq_ws_num_params": ([], C.c_longlong),
    "idq_ws_get_params": ([vp, dp], ip),
    "idq_ws_set_params": ([vp, dp], ip),
    "idq_ws_forward": ([vp, vp, vp, ip, ip, ip, ip, ip, vp], ip),
    "idq_ws_train_step": ([vp, vp, vp, ip, ip, ip, ip, ip, C.c_double, dp, vp], ip),
    "idq_ws_grad": ([vp, vp, vp, vp, ip, ip, ip, ip, ip, dp, vp], ip),
}


class IDQError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libidq error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library (raises if libidq.so was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_19705_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(code, allow=(IDQ_OK,)):
    if code in allow:
        return code
    msg = lib().idq_last_error().decode(errors="replace")
    raise IDQError(code, msg)
