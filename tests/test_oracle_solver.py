"""Pins for oracle.solver (Alg. 1): exact two-root trajectories of both
momentum forms on separable quadratics, the stopping index, restart indices,
the averaging step, the per-frequency closed form of g = 0 with a circular
blur, the dense solve of the linear-network case, and the power iteration
against a dense eigen-decomposition."""
import math

import numpy as np
import pytest

import synth
from oracle import operators as O, regularizer as R, solver as S, backward as B

from test_oracle_operators import fft_correlate
from test_oracle_regularizer import dense_linear_net


def closed_form_errors(mu, beta, tau, e0, K, form):
    """e_k = a r1^k + b r2^k for k = 0..K with e_{-1} = e_0 (complex roots allowed)."""
    q = 1.0 - tau * mu
    if form == "extrapolated":
        s, p = (1 + beta) * q, beta * q
    else:
        s, p = 1 + beta - tau * mu, beta
    disc = np.sqrt(np.asarray(s * s - 4 * p, dtype=complex))
    r1, r2 = (s + disc) / 2, (s - disc) / 2
    e1 = q * e0                      # first step has no inertia in both forms
    a = (e1 - r2 * e0) / (r1 - r2)
    b = e0 - a
    ks = np.arange(K + 1)[:, None]
    return np.real(a * r1 ** ks + b * r2 ** ks)


@pytest.mark.parametrize("form", ["extrapolated", "current"])
@pytest.mark.parametrize("beta", [0.0, 0.5, 0.8])
def test_quadratic_trajectory_exact(form, beta):
    mu = np.array([0.05, 0.3, 1.0, 1.7, 2.0])
    c = np.array([0.3, -1.0, 2.0, 0.5, 0.0])
    x0 = np.array([1.0, 2.0, -1.0, 0.0, 3.0])
    tau = 0.9 / 2.0
    E = closed_form_errors(mu, beta, tau, x0 - c, 40, form)
    grad = lambda p, idx: mu * (p - c)
    for K in (1, 2, 3, 7, 40):
        xk, info = S.inertial_iterate(x0[None], grad, beta, tau, fixed_iters=K, grad_at=form)
        np.testing.assert_allclose(xk[0], c + E[K], atol=1e-12)
        assert info["iters"][0] == K and info["status"][0] == S.FIXED


def test_momentum_rate_is_sqrt_beta_q():
    # complex-root regime: |r| = sqrt(beta q) for the extrapolated form
    beta, tau, mu = 0.5, 0.45, 1.0
    E = closed_form_errors(np.array([mu]), beta, tau, np.array([1.0]), 200, "extrapolated")
    q = 1 - tau * mu
    assert (1 + beta) ** 2 * q * q < 4 * beta * q
    env = np.abs(E[150:, 0]).max() / np.abs(E[50:100, 0]).max()
    assert env < (beta * q) ** (0.5 * 50) * 10


def test_stopping_index_matches_closed_form():
    mu = np.array([0.2, 1.0, 1.9])
    c = np.array([1.0, 1.0, 1.0])
    x0 = np.array([2.0, 0.0, 1.5])
    beta, tau = 0.5, 0.45
    E = closed_form_errors(mu, beta, tau, x0 - c, 400, "extrapolated")
    X = c + E
    rel = np.linalg.norm(X[1:] - X[:-1], axis=1) / np.linalg.norm(X[:-1], axis=1)
    k_stop = int(np.argmax(rel < 1e-6)) + 1
    xk, info = S.inertial_iterate(x0[None], lambda p, i: mu * (p - c), beta, tau, tol=1e-6, max_iter=1000)
    assert info["iters"][0] == k_stop and info["status"][0] == S.CONVERGED
    np.testing.assert_allclose(xk[0], X[k_stop], atol=1e-12)


def test_restart_indices_against_closed_form_segments():
    mu, beta, tau, B2 = 1.0, 0.8, 0.5, 0.5
    x0, K = 3.0, 60
    grad = lambda p, idx: mu * p
    # expected: piecewise closed-form trajectories, each segment restarting with e_{-1} = e_0
    expected, traj = [], [x0]
    start, it = x0, 0
    while it < K:
        E = closed_form_errors(np.array([mu]), beta, tau, np.array([start]), K, "extrapolated")[:, 0]
        Ssum = 0.0
        for j in range(1, K + 1):
            Ssum += (E[j] - E[j - 1]) ** 2
            it += 1
            traj.append(E[j])
            if j * Ssum > B2:
                expected.append(it)
                start = E[j]
                break
            if it >= K:
                break
    xk, info = S.inertial_iterate(np.array([[x0]]), grad, beta, tau, fixed_iters=K,
                                  restart_B=math.sqrt(B2), record=True)
    assert info["restart_at"][0] == expected and len(expected) >= 2
    np.testing.assert_allclose(xk[0, 0], traj[K], atol=1e-12)


def test_averaging_step_closed_form():
    mu = np.array([0.3, 1.2])
    c = np.array([0.5, -0.5])
    x0 = np.array([1.0, 1.0])
    beta, tau, K = 0.6, 0.5, 20
    X = c + closed_form_errors(mu, beta, tau, x0 - c, K, "extrapolated")
    Xm1 = np.vstack([X[:1], X[:-1]])                     # x^{k-1} with x^{-1} = x^0
    Z = X + beta * (X - Xm1)                             # z^k
    steps = np.linalg.norm(X[1:] - X[:-1], axis=1)        # ||x^{k+1} - x^k||
    ks = [k for k in range(K // 2 + 1, K - 1)]
    K0 = ks[int(np.argmin(steps[ks]))]
    want = Z[:K0 + 1].mean(axis=0)
    got, _ = S.inertial_iterate(x0[None], lambda p, i: mu * (p - c), beta, tau,
                                fixed_iters=K, averaging=True)
    np.testing.assert_allclose(got[0], want, atol=1e-13)


def test_g0_identity_converges_to_y(rng):
    y = rng.uniform(0, 1, (2, 3, 5, 4))
    P = S.Problem(O.Operator("identity"), None, 0.0)
    x, info = S.ideq_solve(P, y, np.zeros_like(y), 0.5, 0.9, tol=1e-14, max_iter=500)
    np.testing.assert_allclose(x, y, atol=1e-12)
    assert np.all(info["status"] == S.CONVERGED)


def test_g0_blur_kth_iterate_by_fourier_matrix_power(rng):
    k = synth.gaussian_taps(9, 1.6)
    h, w, beta, K = 12, 10, 0.5, 25
    tau = 0.9
    y = rng.uniform(0, 1, (1, 1, h, w))
    x0 = rng.uniform(0, 1, (1, 1, h, w))
    P = S.Problem(O.Operator("blur", k), None, 0.0)
    xk, _ = S.ideq_solve(P, y, x0, beta, tau, fixed_iters=K)
    kap = np.zeros((h, w))
    for a in range(9):
        for b in range(9):
            kap[(a - 4) % h, (b - 4) % w] += k[a, b]
    Kh = np.fft.fft2(kap)
    Y, X0 = np.fft.fft2(y[0, 0]), np.fft.fft2(x0[0, 0])
    XK = np.empty((h, w), dtype=complex)
    for i in range(h):
        for j in range(w):
            q = 1.0 - tau * abs(Kh[i, j]) ** 2
            M = np.array([[(1 + beta) * q, -beta * q, tau * Kh[i, j] * Y[i, j]],
                          [1, 0, 0], [0, 0, 1]], dtype=complex)
            s = np.linalg.matrix_power(M, K) @ np.array([X0[i, j], X0[i, j], 1.0])
            XK[i, j] = s[0]
    np.testing.assert_allclose(xk[0, 0], np.real(np.fft.ifft2(XK)), atol=1e-12)


def dense_blur(k, h, w):
    kh, kw = k.shape
    ry, rx = (kh - 1) // 2, (kw - 1) // 2
    A = np.zeros((h * w, h * w))
    for i in range(h):
        for j in range(w):
            for a in range(kh):
                for b in range(kw):
                    A[i * w + j, ((i + a - ry) % h) * w + (j + b - rx) % w] += k[a, b]
    return A


def test_linear_network_fixed_point_is_dense_solve(rng):
    h, w, lam = 8, 7, 0.7
    # weights scaled down so that M = I - W_eff is well conditioned
    layers = [(0.2 * W, b) for W, b in synth.he_normal_net([1, 4, 1], 5, bias_seed=9)]
    net = R.Net(layers, act="identity")
    k = synth.gaussian_taps(5, 1.0)
    A = dense_blur(k, h, w)
    Weff, c0 = dense_linear_net(layers, 1, h, w)
    M = np.eye(h * w) - Weff
    Hd = A.T @ A + lam * M.T @ M
    ev = np.linalg.eigvalsh(Hd)
    assert ev[0] > 0.3
    y = rng.uniform(0, 1, (1, 1, h, w))
    xstar = np.linalg.solve(Hd, A.T @ y.ravel() + lam * M.T @ c0)
    P = S.Problem(O.Operator("blur", k), net, lam)
    x, info = S.ideq_solve(P, y, y, 0.5, 0.9 / ev[-1], tol=1e-14, max_iter=20000)
    assert info["status"][0] == S.CONVERGED
    np.testing.assert_allclose(x.ravel(), xstar, atol=1e-11)


def test_power_iteration_against_dense_eigenvalues():
    net = R.Net(synth.he_normal_net(synth.net_channels("gray16"), 0))
    xt, nz = synth.make_batch(1, 1, 1, 6, 6)
    y = xt + 25 / 255 * nz
    P = S.Problem(O.Operator("identity"), net, 1.0)
    H = B.dense_hessian(P, y, y)
    np.testing.assert_allclose(H, H.T, atol=1e-12)
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    top = ev[np.argmax(np.abs(ev))]
    v0 = synth.random_field(12345, y.shape)
    L_long = S.power_iteration(P, y, y, v0, iters=3000)
    assert abs(L_long - top) < 1e-8 * abs(top)
    L30 = S.power_iteration(P, y, y, v0, iters=30)
    assert 0.8 * abs(top) < L30 <= abs(top) * (1 + 1e-12)
