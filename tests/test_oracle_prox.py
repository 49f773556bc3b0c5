"""Pins for the inpainting and MRI operators (App. D.3.1-2), the proximal step
of f (App. B, eq. red_prox) and the i-DEQ-P iteration (Alg. 2):
  * the MRI operator against an explicit DFT matrix, its adjoint by the dot
    test for the real inner product, the unitary norm;
  * every closed-form prox against a dense solve of its normal equations
    (I + tau A^T A) x = v + tau A^T y, with A^T A assembled column by column;
  * the prox as the minimiser: the gradient of the prox objective vanishes;
  * i-DEQ-P with g = 0: the exact K-th iterate of the per-pixel / per-frequency
    linear recurrence;
  * i-DEQ-P with a linear network: its fixed point is the dense minimiser of
    f + lambda g, as for Alg. 1.
"""
import numpy as np
import pytest

import synth
from oracle import operators as O, regularizer as R, solver as S

from test_oracle_regularizer import dense_linear_net


def dft_matrix(n):
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n) / np.sqrt(n)


def make_op(kind, h, w, seed=3):
    rng = np.random.default_rng(seed)
    if kind == "identity":
        return O.Operator("identity")
    if kind == "inpaint":
        return O.Operator("inpaint", mask=synth.pixel_mask(seed, h, w, 0.5))
    if kind == "blur":
        return O.Operator("blur", rng.uniform(0, 1, (5, 3)))      # asymmetric taps
    if kind == "mri_random":                                     # no k -> -k symmetry
        return O.Operator("mri", mask=(rng.random((h, w)) < 0.4).astype(float))
    if kind == "mri_cartesian":
        return O.Operator("mri", mask=synth.cartesian_mask(seed, h, w, accel=4))
    raise ValueError(kind)


def measurement(op, shape, rng):
    x = rng.uniform(0, 1, shape)
    y = op.A(x)
    if np.iscomplexobj(y):
        return y + 0.05 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    return y + 0.05 * rng.standard_normal(shape)


def test_mri_operator_is_the_masked_unitary_dft(rng):
    h, w = 8, 6
    op = make_op("mri_random", h, w)
    x = rng.standard_normal((2, 3, h, w))
    Fh, Fw = dft_matrix(h), dft_matrix(w)
    want = op.mask * np.einsum("ab,ncbd,ed->ncae", Fh, x, Fw)
    np.testing.assert_allclose(op.A(x), want, atol=1e-13)
    full = O.Operator("mri", mask=np.ones((h, w)))
    np.testing.assert_allclose(np.sum(np.abs(full.A(x)) ** 2), np.sum(x * x), rtol=1e-13)
    v = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
    lhs = np.sum(np.real(np.conj(op.A(x)) * v))
    rhs = np.sum(x * op.vjp(None, v))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("kind", ["inpaint", "mri_random", "mri_cartesian"])
def test_mask_operator_gradient_by_central_differences(kind, rng):
    h, w = 8, 8
    op = make_op(kind, h, w)
    y = measurement(op, (1, 2, h, w), rng)
    x = rng.standard_normal((1, 2, h, w))
    d = rng.standard_normal(x.shape)
    e = 1e-6
    fd = (op.f(x + e * d, y) - op.f(x - e * d, y)) / (2 * e)
    np.testing.assert_allclose(fd, np.sum(op.grad_f(x, y) * d, axis=(1, 2, 3)), rtol=1e-8)
    np.testing.assert_allclose(op.hess_f(x, y, d), op.vjp(None, op.jvp(None, d)), atol=1e-14)


def dense_normal_matrix(op, shape):
    d = int(np.prod(shape))
    G = np.zeros((d, d))
    e = np.zeros(d)
    for i in range(d):
        e[:] = 0.0
        e[i] = 1.0
        G[:, i] = op.vjp(None, op.jvp(None, e.reshape(shape))).ravel()
    return G


@pytest.mark.parametrize("kind", ["identity", "inpaint", "blur", "mri_random", "mri_cartesian"])
@pytest.mark.parametrize("tau", [0.3, 2.5])
def test_prox_is_the_dense_solve(kind, tau, rng):
    shape = (1, 1, 8, 6)
    op = make_op(kind, *shape[-2:])
    y = measurement(op, shape, rng)
    v = rng.standard_normal(shape)
    G = dense_normal_matrix(op, shape)
    rhs = v.ravel() + tau * op.vjp(None, y).ravel()
    want = np.linalg.solve(np.eye(G.shape[0]) + tau * G, rhs)
    got = op.prox(v, y, tau)
    assert got.dtype == np.float64
    np.testing.assert_allclose(got.ravel(), want, atol=1e-12)
    # optimality of the prox objective 1/2 ||A x - y||^2 + ||x - v||^2 / (2 tau)
    np.testing.assert_allclose(op.grad_f(got, y) + (got - v) / tau, 0.0, atol=1e-11)


def test_paper_inpainting_prox_leaves_missing_pixels():
    op = make_op("inpaint", 6, 5)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((1, 3, 6, 5))
    y = rng.standard_normal((1, 3, 6, 5))
    p = op.prox(v, y, 0.7)
    miss = op.mask == 0
    np.testing.assert_array_equal(p[..., miss], v[..., miss])


def test_rician_and_tanh_have_no_closed_form_prox():
    for op in (O.Operator("rician", sigma=0.1), O.Operator("tanh_blur", np.ones((3, 3)) / 9)):
        with pytest.raises(ValueError):
            op.prox(np.zeros((1, 1, 4, 4)), np.zeros((1, 1, 4, 4)), 0.5)


@pytest.mark.parametrize("beta", [0.0, 0.5, 0.9])
def test_ideq_p_g0_inpainting_kth_iterate(beta, rng):
    """Observed pixels follow e_{k+1} = ((1 + beta) e_k - beta e_{k-1}) / (1 + tau)
    for e = x - y; missing pixels never move (x^{-1} = x^0)."""
    h, w, tau, K = 6, 5, 0.8, 17
    op = make_op("inpaint", h, w)
    y = rng.uniform(0, 1, (1, 2, h, w))
    x0 = rng.uniform(0, 1, (1, 2, h, w))
    P = S.Problem(op, None, 0.0)
    xk, info = S.ideq_solve(P, y, x0, beta, tau, proximal=True, fixed_iters=K)
    e_prev = e = x0 - y
    for _ in range(K):
        e, e_prev = ((1 + beta) * e - beta * e_prev) / (1 + tau), e
    want = np.where(op.mask == 1, y + e, x0)
    np.testing.assert_allclose(xk, want, atol=1e-13)
    assert info["status"][0] == S.FIXED


def test_ideq_p_g0_blur_kth_iterate_by_fourier_matrix_power(rng):
    k = synth.gaussian_taps(5, 1.0)
    h, w, beta, tau, K = 8, 10, 0.5, 1.7, 23
    op = O.Operator("blur", k)
    y = rng.uniform(0, 1, (1, 1, h, w))
    x0 = rng.uniform(0, 1, (1, 1, h, w))
    xk, _ = S.ideq_solve(S.Problem(op, None, 0.0), y, x0, beta, tau, proximal=True,
                         fixed_iters=K)
    kap = np.zeros((h, w))
    for a in range(5):
        for b in range(5):
            kap[(a - 2) % h, (b - 2) % w] += k[a, b]
    Kh = np.fft.fft2(kap)
    Y, X0 = np.fft.fft2(y[0, 0]), np.fft.fft2(x0[0, 0])
    XK = np.empty((h, w), dtype=complex)
    for i in range(h):
        for j in range(w):
            d = 1.0 + tau * abs(Kh[i, j]) ** 2
            M = np.array([[(1 + beta) / d, -beta / d, tau * np.conj(Kh[i, j]) * Y[i, j] / d],
                          [1, 0, 0], [0, 0, 1]], dtype=complex)
            XK[i, j] = (np.linalg.matrix_power(M, K) @ np.array([X0[i, j], X0[i, j], 1.0]))[0]
    np.testing.assert_allclose(xk[0, 0], np.real(np.fft.ifft2(XK)), atol=1e-12)


@pytest.mark.parametrize("kind", ["inpaint", "mri_cartesian"])
def test_ideq_p_linear_network_fixed_point_is_dense_minimiser(kind, rng):
    h, w, lam = 8, 8, 0.7
    layers = [(0.2 * W, b) for W, b in synth.he_normal_net([1, 4, 1], 5, bias_seed=9)]
    net = R.Net(layers, act="identity")
    op = make_op(kind, h, w)
    Weff, c0 = dense_linear_net(layers, 1, h, w)
    M = np.eye(h * w) - Weff
    G = dense_normal_matrix(op, (1, 1, h, w))
    Hd = G + lam * M.T @ M
    assert np.linalg.eigvalsh(Hd)[0] > 0.05
    y = measurement(op, (1, 1, h, w), rng)
    xstar = np.linalg.solve(Hd, op.vjp(None, y).ravel() + lam * M.T @ c0)
    Lg = np.linalg.eigvalsh(lam * M.T @ M)[-1]
    x, info = S.ideq_solve(S.Problem(op, net, lam), y, op.vjp(None, y), 0.5, 0.9 / Lg,
                           proximal=True, tol=1e-14, max_iter=20000)
    assert info["status"][0] == S.CONVERGED
    np.testing.assert_allclose(x.ravel(), xstar, atol=1e-11)


def test_ideq_p_rejects_the_current_point_form():
    P = S.Problem(O.Operator("identity"), None, 0.0)
    with pytest.raises(ValueError):
        S.ideq_solve(P, np.zeros((1, 1, 2, 2)), np.zeros((1, 1, 2, 2)), 0.5, 0.5,
                     proximal=True, grad_at="current", fixed_iters=2)
