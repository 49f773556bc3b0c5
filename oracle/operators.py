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
  inpaint       A(x) = M . x, M an (h, w) 0/1 pixel mask applied to every
                channel (App. D.3.2)
  mri           A(x) = M . F x with F the unitary 2-D DFT of each plane and M
                an (h, w) 0/1 k-space mask; x is real (the phase is fixed to
                zero, App. D.3.1) and y complex (n, c, h, w)
  rician        the Rician likelihood of App. D.3.3 instead of a Gaussian one:
                f(x, y) = sum x^2 / (2 s^2) - log I_0(x y / s^2), s = sigma_y

For real x and complex data the inner product is Re<u, v>, so the adjoint of
x -> M F x is v -> Re(F^H (M v)) and grad f = Re(F^H M (M F x - y)).

Proximal step (App. B, eq. red_prox, and the closed forms of App. D.3.1-2):
for a linear A, prox_{tau f}(v) = argmin_x 1/2 ||A x - y||^2 + ||x - v||^2 / (2 tau)
solves (I + tau A^T A) x = v + tau A^T y.  A^T A is diagonal for the
inpainting mask (the paper's (tau M y + v) / (tau M + 1)), and diagonalised by
the DFT for the circular blur (multiplier |k^|^2) and for the real-valued MRI
problem (multiplier M_s(k) = (M(k) + M(-k)) / 2, the real part of F^H M F on
real images; M_s = M for a mask symmetric under k -> -k).  Those
diagonalisations are what ``prox`` evaluates; the pin solves the same linear
system densely (tests/test_oracle_prox.py).

Circular correlation with a kh x kw tap array k centred at (ry, rx):
  (B x)[i, j] = sum_{a,b} k[a, b] x[(i + a - ry) mod h, (j + b - rx) mod w].
Pins: FFT evaluation of B (correlation theorem), adjoint dot tests, central
differences of A for the Jacobian products (tests/test_oracle_operators.py).
"""
import numpy as np

from .bessel import log_i0, ratio, ratio_derivative


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


def _wrapped_taps(k, h, w):
    """The taps of B placed on an h x w grid at their circular offsets, so that
    B x = ifft2(fft2(x) * conj(fft2(kap))) (correlation theorem)."""
    kh, kw = k.shape
    ry, rx = (kh - 1) // 2, (kw - 1) // 2
    kap = np.zeros((h, w))
    for a in range(kh):
        for b in range(kw):
            kap[(a - ry) % h, (b - rx) % w] += k[a, b]
    return kap


def symmetrised_mask(m):
    """M_s(k) = (M(k) + M(-k)) / 2 on the FFT index grid (-k taken mod h, w)."""
    flip = np.roll(m[::-1, ::-1], shift=(1, 1), axis=(0, 1))
    return 0.5 * (m + flip)


class Operator:
    """A forward model with A(x), J_A(x) w, J_A(x)^T v and the second-order
    term of f's Hessian.

    kind: 'identity' | 'blur' | 'tanh_blur' | 'inpaint' | 'mri' | 'rician';
    ``taps`` for the blurs; ``gain`` is gamma of the tanh-blur (2 in the
    nonlinear workload); ``mask`` (h, w) for inpainting and MRI; ``sigma`` the
    Rician noise level sigma_y.
    """

    def __init__(self, kind, taps=None, gain=2.0, mask=None, sigma=None):
        self.kind = kind
        self.k = None if taps is None else np.asarray(taps, dtype=np.float64)
        self.gain = float(gain)
        self.mask = None if mask is None else np.asarray(mask, dtype=np.float64)
        self.sigma = None if sigma is None else float(sigma)
        if kind in ("blur", "tanh_blur") and self.k is None:
            raise ValueError("blur operators need taps")
        if kind in ("inpaint", "mri") and self.mask is None:
            raise ValueError("mask operators need a mask")
        if kind == "rician" and not (self.sigma and self.sigma > 0):
            raise ValueError("the Rician term needs sigma > 0")

    # ---- A and its derivatives -------------------------------------------
    def A(self, x):
        if self.kind in ("identity", "rician"):
            return x.copy()
        if self.kind == "inpaint":
            return self.mask * x
        if self.kind == "mri":
            return self.mask * np.fft.fft2(x, norm="ortho")
        bx = blur(x, self.k)
        if self.kind == "blur":
            return bx
        g = self.gain
        return np.tanh(g * bx) / np.tanh(g)

    def jvp(self, x, w):
        """J_A(x) w."""
        if self.kind in ("identity", "rician"):
            return w.copy()
        if self.kind in ("inpaint", "mri"):
            return self.A(w)
        if self.kind == "blur":
            return blur(w, self.k)
        g = self.gain
        t = np.tanh(g * blur(x, self.k))
        return (g / np.tanh(g)) * (1.0 - t * t) * blur(w, self.k)

    def vjp(self, x, v):
        """J_A(x)^T v (x is ignored for the linear operators)."""
        if self.kind in ("identity", "rician"):
            return v.copy()
        if self.kind == "inpaint":
            return self.mask * v
        if self.kind == "mri":
            return np.real(np.fft.ifft2(self.mask * v, norm="ortho"))
        if self.kind == "blur":
            return blur_adjoint(v, self.k)
        g = self.gain
        t = np.tanh(g * blur(x, self.k))
        return blur_adjoint((g / np.tanh(g)) * (1.0 - t * t) * v, self.k)

    # ---- data term ----------------------------------------------------------
    def f(self, x, y):
        """Per-image value of f, shape (n,): 1/2 ||A(x) - y||^2, or the Rician
        negative log-likelihood up to its constant."""
        if self.kind == "rician":
            s2 = self.sigma ** 2
            return np.sum(x * x / (2.0 * s2) - log_i0(x * y / s2), axis=(1, 2, 3))
        r = self.A(x) - y
        return 0.5 * np.sum(np.real(r * np.conj(r)), axis=(1, 2, 3))

    def grad_f(self, x, y):
        """grad_x f = J_A(x)^T (A(x) - y); for the Rician term
        x / s^2 - (y / s^2) B(x y / s^2) with B = I_1 / I_0."""
        if self.kind == "rician":
            s2 = self.sigma ** 2
            return x / s2 - (y / s2) * ratio(x * y / s2)
        return self.vjp(x, self.A(x) - y)

    def hess_f(self, x, y, w):
        """Hessian of f along w: J_A^T J_A w plus, for the tanh-blur, the
        curvature of A weighted by the residual:
        B^T[(A(x) - y) * (-2 gamma^2 / tanh(gamma)) t (1 - t^2) * (B w)],
        t = tanh(gamma B x).  The Rician Hessian is diagonal:
        1 / s^2 - (y / s^2)^2 B'(x y / s^2)."""
        if self.kind == "rician":
            s2 = self.sigma ** 2
            return (1.0 / s2 - (y / s2) ** 2 * ratio_derivative(x * y / s2)) * w
        gn = self.vjp(x, self.jvp(x, w))
        if self.kind != "tanh_blur":
            return gn
        g = self.gain
        bx = blur(x, self.k)
        t = np.tanh(g * bx)
        res = np.tanh(g * bx) / np.tanh(g) - y
        curv = (-2.0 * g * g / np.tanh(g)) * t * (1.0 - t * t)
        return gn + blur_adjoint(res * curv * blur(w, self.k), self.k)

    # ---- proximal step (App. B) ---------------------------------------------
    def prox(self, v, y, tau):
        """prox_{tau f(., y)}(v) = (I + tau A^T A)^{-1} (v + tau A^T y) for the
        linear operators; the Rician and tanh-blur terms have no closed form."""
        rhs = v + tau * self.vjp(None, y)
        if self.kind == "identity":
            return rhs / (1.0 + tau)
        if self.kind == "inpaint":
            return rhs / (1.0 + tau * self.mask)
        h, w = v.shape[-2:]
        if self.kind == "blur":
            mult = np.abs(np.fft.fft2(_wrapped_taps(self.k, h, w))) ** 2
        elif self.kind == "mri":
            mult = symmetrised_mask(self.mask)
        else:
            raise ValueError(f"no closed-form proximal step for {self.kind}")
        return np.real(np.fft.ifft2(np.fft.fft2(rhs) / (1.0 + tau * mult)))
