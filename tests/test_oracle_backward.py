"""Pins for oracle.backward on a standalone 3x8x8 deblurring problem (9x9 taps
alias on the 8x8 torus): the dense-Hessian solve of the adjoint equation,
central differences of the loss through tightly re-solved fixed points (the
implicit gradient), and the JFB closed form."""
import math

import numpy as np
import pytest

import synth
from oracle import operators as O, regularizer as R, solver as S, backward as B


@pytest.fixture(scope="module")
def crop_problem():
    net = R.Net(synth.he_normal_net(synth.net_channels("rgb64"), 0))
    op = O.Operator("blur", synth.gaussian_taps(9, 1.6))
    xt, nz = synth.make_batch(4, 1, 3, 8, 8)
    y = op.A(xt) + 0.01 * nz
    P = S.Problem(op, net, 1.0)
    L = S.power_iteration(P, y, y, synth.random_field(12345, y.shape), 30)
    tau = 0.9 / L
    xbar, info = S.ideq_solve(P, y, y, 0.5, tau, tol=1e-14, max_iter=20000)
    assert info["status"][0] == S.CONVERGED
    H = B.dense_hessian(P, xbar, y)
    return dict(P=P, y=y, xt=xt, tau=tau, xbar=xbar, H=0.5 * (H + H.T), Hraw=H)


def test_fixed_point_is_critical_point(crop_problem):
    c = crop_problem
    g = c["P"].grad(c["xbar"], c["y"])
    assert np.max(np.abs(g)) < 1e-10
    np.testing.assert_allclose(c["Hraw"], c["Hraw"].T, atol=1e-10)
    assert np.linalg.eigvalsh(c["H"])[0] > 0          # a local minimum


def test_adjoint_iteration_matches_dense_solve(crop_problem, rng):
    c = crop_problem
    v = rng.standard_normal(c["xbar"].shape)
    u_dense = np.linalg.solve(c["tau"] * c["H"], v.ravel()).reshape(v.shape)
    ev = np.linalg.eigvalsh(c["tau"] * c["H"])
    assert 0 < ev[0] and ev[-1] < 2
    u, iters, rel = B.adjoint_iterate(c["P"], c["xbar"], c["y"], v, c["tau"],
                                      max_iter=200000, tol=1e-14)
    np.testing.assert_allclose(u, u_dense, atol=1e-8 * np.max(np.abs(u_dense)))
    u2, it2, _ = B.adjoint_iterate(c["P"], c["xbar"], c["y"], v, c["tau"],
                                   max_iter=200000, tol=1e-14, beta=0.5)
    np.testing.assert_allclose(u2, u_dense, atol=1e-8 * np.max(np.abs(u_dense)))
    assert it2 < iters


def test_implicit_gradient_by_central_differences(crop_problem, rng):
    c = crop_problem
    P, y, tau = c["P"], c["y"], c["tau"]
    xstar = c["xt"]
    loss = lambda x: 0.5 * np.sum((x - xstar) ** 2)
    v = c["xbar"] - xstar
    u = np.linalg.solve(tau * c["H"], v.ravel()).reshape(v.shape)
    dtheta, dlam = B.theta_grad(P, c["xbar"], y, u, tau)
    p = P.net.pack()

    def solve_with(net, lam):
        Pp = S.Problem(P.op, net, lam)
        x, info = S.ideq_solve(Pp, y, c["xbar"], 0.5, tau, tol=1e-15, max_iter=50000)
        return x

    d = rng.standard_normal(p.size)
    d /= np.linalg.norm(d)
    eps = 1e-4
    lp = loss(solve_with(P.net.with_params(p + eps * d), P.lam))
    lm = loss(solve_with(P.net.with_params(p - eps * d), P.lam))
    fd = (lp - lm) / (2 * eps)
    assert abs(fd - np.dot(dtheta, d)) < 1e-5 * max(abs(fd), 1e-8) + 1e-10
    lp = loss(solve_with(P.net, P.lam + eps))
    lm = loss(solve_with(P.net, P.lam - eps))
    fd = (lp - lm) / (2 * eps)
    assert abs(fd - dlam) < 1e-5 * abs(fd) + 1e-10


def test_jfb_closed_form(crop_problem, rng):
    c = crop_problem
    P, tau = c["P"], c["tau"]
    v = rng.standard_normal(c["xbar"].shape)
    dtheta, dlam = B.theta_grad(P, c["xbar"], c["y"], v, tau)
    p = P.net.pack()
    d = rng.standard_normal(p.size)
    d /= np.linalg.norm(d)
    eps = 1e-4
    # (dT/dtheta)^T v = -tau lam d/dtheta <v, grad g>
    fp = np.sum(v * P.net.with_params(p + eps * d).grad(c["xbar"]))
    fm = np.sum(v * P.net.with_params(p - eps * d).grad(c["xbar"]))
    fd = -tau * P.lam * (fp - fm) / (2 * eps)
    assert abs(fd - np.dot(dtheta, d)) < 1e-7 * abs(fd)
    assert abs(dlam + tau * np.sum(P.net.grad(c["xbar"]) * v)) < 1e-12 * abs(dlam)
