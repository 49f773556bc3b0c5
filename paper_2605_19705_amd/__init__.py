"""i-DEQ inertial fixed-point solver for AMD MI355X (gfx950).

The hot path -- inertial extrapolation, the data-fidelity gradient through the
forward operator A, the learned regularizer's gradient (conv-net forward plus
its vector-Jacobian product) and the fused update / residual / stopping test --
runs in hand-written HIP kernels behind the C ABI of ``include/idq.h``
(``libidq.so``).  This package is the thin Python binding of that ABI.
"""
from . import _lib
from ._lib import IDQError, lib
from .api import IDQ, IDQSolve, SolveResult, Trainer, WarmStart, pack_layers

__all__ = ["IDQ", "IDQSolve", "SolveResult", "Trainer", "WarmStart", "IDQError", "lib", "pack_layers", "_lib"]
