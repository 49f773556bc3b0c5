"""Plain CPU float64 oracle for the i-DEQ hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, links or calls
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library: it is written from the paper's definitions with NumPy, one step
at a time, so it can be checked against the paper by eye.

Modules
  conv         3x3 "same" convolution, its adjoint, its weight gradient, softplus
  operators    forward operators A (identity, circular blur, tanh-blur) and f
  regularizer  gradient-step potential g = 1/2 ||x - N(x)||^2: value, gradient,
               Hessian-vector product and parameter gradients
  solver       the inertial fixed-point iteration (Alg. 1) and the power
               iteration for the step size
  backward     JFB and implicit-differentiation gradients (App. D.1)
  warmstart    the warm-start encoder-decoder (forward, backward, Adam)

Parity status of each function is stated in its docstring; a function with no
independent pin says "parity unpinned".
"""
from . import conv, operators, regularizer, solver, backward, warmstart  # noqa: F401
