"""Pins for oracle.operators: circular blur against the FFT correlation theorem
(with an asymmetric kernel and taps that alias on a small image), adjointness,
and central differences of the nonlinear operator."""
import numpy as np
import pytest

import synth
from oracle import operators as O


def fft_correlate(x, k):
    h, w = x.shape[-2:]
    kh, kw = k.shape
    ry, rx = (kh - 1) // 2, (kw - 1) // 2
    kap = np.zeros((h, w))
    for a in range(kh):
        for b in range(kw):
            kap[(a - ry) % h, (b - rx) % w] += k[a, b]
    K = np.fft.fft2(kap)
    return np.real(np.fft.ifft2(np.fft.fft2(x) * np.conj(K)))


@pytest.mark.parametrize("shape,ks", [((2, 3, 16, 12), (9, 9)), ((1, 3, 8, 8), (9, 9)),
                                      ((1, 1, 7, 5), (3, 5)), ((1, 2, 5, 6), (7, 7))])
def test_blur_equals_fft_correlation(rng, shape, ks):
    x = rng.standard_normal(shape)
    k = rng.standard_normal(ks)            # asymmetric on purpose
    np.testing.assert_allclose(O.blur(x, k), fft_correlate(x, k), atol=1e-12)


def test_blur_adjoint_dot(rng):
    x = rng.standard_normal((2, 3, 10, 8))
    v = rng.standard_normal((2, 3, 10, 8))
    k = rng.standard_normal((9, 9))
    lhs = np.sum(O.blur(x, k) * v)
    rhs = np.sum(x * O.blur_adjoint(v, k))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_gaussian_blur_properties(rng):
    k = synth.gaussian_taps(9, 1.6)
    ones = np.ones((1, 3, 12, 12))
    np.testing.assert_allclose(O.blur(ones, k), ones, atol=1e-14)   # A 1 = 1
    x = rng.standard_normal((1, 3, 12, 12))
    np.testing.assert_allclose(O.blur(x, k), O.blur_adjoint(x, k), atol=1e-14)  # A^T = A
    # Lipschitz constant of grad f = max |k_hat|^2 = 1 (value at frequency 0)
    kap = np.zeros((32, 32))
    kap[:9, :9] = k
    assert abs(np.max(np.abs(np.fft.fft2(kap))) ** 2 - 1.0) < 1e-12


@pytest.mark.parametrize("kind", ["identity", "blur", "tanh_blur"])
def test_jacobians_by_central_differences(rng, kind):
    taps = None if kind == "identity" else rng.uniform(0.0, 1.0, (7, 7)) / 20.0
    op = O.Operator(kind, taps)
    x = rng.uniform(0, 1, (2, 3, 9, 10))
    y = rng.uniform(0, 1, (2, 3, 9, 10))
    w = rng.standard_normal(x.shape)
    v = rng.standard_normal(x.shape)
    eps = 1e-5
    jvp_fd = (op.A(x + eps * w) - op.A(x - eps * w)) / (2 * eps)
    np.testing.assert_allclose(op.jvp(x, w), jvp_fd, atol=1e-8)
    assert abs(np.sum(op.jvp(x, w) * v) - np.sum(w * op.vjp(x, v))) < 1e-10 * np.sum(np.abs(w * op.vjp(x, v)))
    # grad f by differences of f, Hessian of f by differences of grad f
    fd = (op.f(x + eps * w, y) - op.f(x - eps * w, y)) / (2 * eps)
    np.testing.assert_allclose(np.sum(op.grad_f(x, y) * w, axis=(1, 2, 3)), fd, rtol=1e-7)
    hfd = (op.grad_f(x + eps * w, y) - op.grad_f(x - eps * w, y)) / (2 * eps)
    np.testing.assert_allclose(op.hess_f(x, y, w), hfd, atol=1e-8)


def test_tanh_blur_definition(rng):
    k = synth.uniform_taps(7)
    op = O.Operator("tanh_blur", k, gain=2.0)
    x = rng.uniform(0, 1, (1, 3, 9, 9))
    np.testing.assert_allclose(op.A(x), np.tanh(2 * fft_correlate(x, k)) / np.tanh(2), atol=1e-13)
    ones = np.ones((1, 1, 9, 9))
    np.testing.assert_allclose(op.A(ones), ones, atol=1e-14)        # A(1) = tanh 2 / tanh 2
