"""Forward operators A and the data-fidelity term f, float64.

The inverse problem is y = A(x) + n with x_hat in argmin f(x, y) + lambda g(x)
(Sec. 1, eq. inv_prob).  For additive Gaussian noise the fidelity is
f(x, y) = 1/2 ||A(x) - y||^2 with gradient J_A(x)^T (A(x) - y); the paper
writes exactly this form for its linear operators (App. D.3.1 and D.3.2, where
grad f = A^T (A x - y) and the Lipschitz constant of grad f is 1 for their
operators).

Operators provided (all act channel-wise on (n, c, h, w) arrays):
  identity      A(x) = x                                     (denoising)
  blur          circular cross-correlation with taps k       (deblurring)
  tanh_blur     A(x) = tanh(gamma * (k * x)) / tanh(gamma)   (nonlinear)

Circular correlation with a kh x kw tap array k centred at (ry, rx):
  (B x)[i, j] = sum_{a,b} k[a, b] x[(i + a - ry) mod h, (j + b - rx) mod w].
Pins: FFT evaluation of B (correlation theorem), adjoint dot tests, central
differences of A for the Jacobian products (tests/test_oracle_operators.py).
"""
import numpy as np


def blur(x, k):
    """Circular cross-correlation B x (definition in the module docstring)."""
    kh, kw = k.shape
    ry, rx = (kh - 1) // 2, (kw - 1) // 2
    out = np.zeros_like(x)
    for a in range(kh):
        for b in range(kw):
            out += k[a, b] * np.roll(x, shift=(-(a - ry), -(b - rx)), axis=(-2, -1))
    return out


def blur_adjoint(v, k):
    """B^T v[i, j] = sum_{a,b} k[a, b] v[(i - a + ry) mod h, (j - b + rx) mod w]."""
    kh, kw = k.shape
    ry, rx = (kh - 1) // 2, (kw - 1) // 2
    out = np.zeros_like(v)
    for a in range(kh):
        for b in range(kw):
            out += k[a, b] * np.roll(v, shift=(a - ry, b - rx), axis=(-2, -1))
    return out


class Operator:
    """A forward model with A(x), J_A(x) w, J_A(x)^T v and the second-order
    term of f's Hessian.

    kind: 'identity' | 'blur' | 'tanh_blur'; ``taps`` for the blurs;
    ``gain`` is gamma of the tanh-blur (2 in the nonlinear workload).
    """

    def __init__(self, kind, taps=None, gain=2.0):
        self.kind = kind
        self.k = None if taps is None else np.asarray(taps, dtype=np.float64)
        self.gain = float(gain)
        if kind != "identity" and self.k is None:
            raise ValueError("blur operators need taps")

    # ---- A and its derivatives -------------------------------------------
    def A(self, x):
        if self.kind == "identity":
            return x.copy()
        bx = blur(x, self.k)
        if self.kind == "blur":
            return bx
        g = self.gain
        return np.tanh(g * bx) / np.tanh(g)

    def jvp(self, x, w):
        """J_A(x) w."""
        if self.kind == "identity":
            return w.copy()
        if self.kind == "blur":
            return blur(w, self.k)
        g = self.gain
        t = np.tanh(g * blur(x, self.k))
        return (g / np.tanh(g)) * (1.0 - t * t) * blur(w, self.k)

    def vjp(self, x, v):
        """J_A(x)^T v (x is ignored for the linear operators)."""
        if self.kind == "identity":
            return v.copy()
        if self.kind == "blur":
            return blur_adjoint(v, self.k)
        g = self.gain
        t = np.tanh(g * blur(x, self.k))
        return blur_adjoint((g / np.tanh(g)) * (1.0 - t * t) * v, self.k)

    # ---- data term f(x, y) = 1/2 ||A(x) - y||^2 ---------------------------
    def f(self, x, y):
        """Per-image value of f, shape (n,)."""
        r = self.A(x) - y
        return 0.5 * np.sum(r * r, axis=(1, 2, 3))

    def grad_f(self, x, y):
        """grad_x f = J_A(x)^T (A(x) - y)."""
        return self.vjp(x, self.A(x) - y)

    def hess_f(self, x, y, w):
        """Hessian of f along w: J_A^T J_A w plus, for the tanh-blur, the
        curvature of A weighted by the residual:
        B^T[(A(x) - y) * (-2 gamma^2 / tanh(gamma)) t (1 - t^2) * (B w)],
        t = tanh(gamma B x)."""
        gn = self.vjp(x, self.jvp(x, w))
        if self.kind != "tanh_blur":
            return gn
        g = self.gain
        bx = blur(x, self.k)
        t = np.tanh(g * bx)
        res = np.tanh(g * bx) / np.tanh(g) - y
        curv = (-2.0 * g * g / np.tanh(g)) * t * (1.0 - t * t)
        return gn + blur_adjoint(res * curv * blur(w, self.k), self.k)
