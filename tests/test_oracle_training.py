"""Pins for oracle.training (the epoch loop of Alg. 1 / Alg. 2):
  * on a linear network (identity activation) and a linear operator the fixed
    point is x*(Theta) = (A^T A + lambda M^T M)^{-1} (A^T y + lambda M^T c0) in
    closed form, so the implicit gradients of the epoch loss must equal central
    differences of the loss through dense solves, for lambda and for a random
    direction in theta, with the forward run long enough to converge; this
    holds for Alg. 1 and for the proximal Alg. 2;
  * JFB for Alg. 2 applies the proximal step's Jacobian (I + tau A^T A)^{-1}
    (a dense solve here);
  * the gradient accumulated over batches equals the whole-dataset gradient;
  * the Adam step moves every parameter with a nonzero gradient by the
    learning rate, against the gradient's sign (Adam's first step).
"""
import numpy as np
import pytest

import synth
from oracle import operators as O, regularizer as R, training as T

from test_oracle_prox import dense_normal_matrix
from test_oracle_regularizer import dense_linear_net

H, W = 6, 5


def setup(kind, seed=0):
    rng = np.random.default_rng(seed)
    layers = [(0.2 * Wt, b) for Wt, b in synth.he_normal_net([1, 3, 1], 5, bias_seed=9)]
    net = R.Net(layers, act="identity")
    if kind == "blur":
        op = O.Operator("blur", synth.gaussian_taps(3, 0.8))
    else:
        op = O.Operator("inpaint", mask=synth.pixel_mask(2, H, W, 0.6))
    Xs = rng.uniform(0, 1, (3, 1, H, W))
    Y = op.A(Xs) + 0.05 * rng.standard_normal(Xs.shape)
    return net, op, Xs, Y


def dense_fixed_point(net, op, lam, y):
    Weff, c0 = dense_linear_net(net.layers, 1, H, W)
    M = np.eye(H * W) - Weff
    G = dense_normal_matrix(op, (1, 1, H, W))
    return np.linalg.solve(G + lam * M.T @ M, op.vjp(None, y).ravel() + lam * M.T @ c0)


def dense_loss(net, op, lam, Y, Xs):
    N, d = Y.shape[0], H * W
    return sum(float(np.sum((dense_fixed_point(net, op, lam, Y[i:i + 1]) - Xs[i].ravel()) ** 2))
               for i in range(N)) / (N * d)


@pytest.mark.parametrize("kind,proximal", [("blur", False), ("inpaint", False), ("inpaint", True)])
def test_implicit_gradients_are_derivatives_of_the_loss(kind, proximal):
    net, op, Xs, Y = setup(kind)
    lam = 0.7
    tr = T.Trainer(net, op, lam, tau=0.3, beta=0.5, K=3000, mode="implicit", proximal=proximal,
                   adjoint_iters=20000, adjoint_tol=1e-14)
    loss, gth, glam = tr.epoch(Y, Xs)
    assert abs(loss - dense_loss(net, op, lam, Y, Xs)) < 1e-12
    e = 1e-5
    fd_lam = (dense_loss(net, op, lam + e, Y, Xs) - dense_loss(net, op, lam - e, Y, Xs)) / (2 * e)
    assert abs(glam - fd_lam) < 1e-7 * max(1.0, abs(fd_lam)), (glam, fd_lam)
    d = np.random.default_rng(3).standard_normal(gth.size)
    th = net.pack()
    fd_th = (dense_loss(net.with_params(th + e * d), op, lam, Y, Xs)
             - dense_loss(net.with_params(th - e * d), op, lam, Y, Xs)) / (2 * e)
    assert abs(float(gth @ d) - fd_th) < 1e-7 * max(1.0, abs(fd_th)), (gth @ d, fd_th)


def test_proximal_jfb_applies_the_prox_jacobian():
    net, op, Xs, Y = setup("inpaint")
    tau, lam = 0.4, 0.8
    tr = T.Trainer(net, op, lam, tau=tau, beta=0.5, K=50, mode="jfb", proximal=True)
    xhat = tr.forward(Y, Y)
    v = np.random.default_rng(5).standard_normal(xhat.shape)
    dt, dl = tr.gradient(xhat, Y, v)
    G = dense_normal_matrix(op, (1, 1, H, W))
    Jp = np.linalg.inv(np.eye(H * W) + tau * G)
    w = np.stack([(Jp @ v[i].ravel()).reshape(v[i].shape) for i in range(v.shape[0])])
    want_l = -tau * float(np.sum(tr.problem().net.grad(xhat) * w))
    assert abs(dl - want_l) < 1e-12 * max(1.0, abs(want_l))
    plain = T.Trainer(net, op, lam, tau=tau, beta=0.5, K=50, mode="jfb", proximal=False)
    dt_w, _ = plain.gradient(xhat, Y, w)           # Alg. 1's JFB with u = J_P v
    np.testing.assert_allclose(dt, dt_w, atol=1e-13)


def test_accumulated_gradient_equals_whole_batch_gradient():
    net, op, Xs, Y = setup("blur")
    kw = dict(tau=0.3, beta=0.5, K=40, mode="jfb", averaging=True)
    a = T.Trainer(net, op, 0.7, **kw)
    b = T.Trainer(net, op, 0.7, **kw)
    la, ga, gla = a.epoch(Y, Xs)
    lb, gb, glb = b.epoch(Y, Xs, batch=1)
    assert abs(la - lb) < 1e-14
    np.testing.assert_allclose(ga, gb, atol=1e-15)
    assert abs(gla - glb) < 1e-15
    np.testing.assert_allclose(a.theta, b.theta, atol=1e-15)


def test_first_adam_step_moves_by_the_learning_rate():
    net, op, Xs, Y = setup("blur")
    lr_t, lr_l = 1e-3, 5e-3
    tr = T.Trainer(net, op, 0.7, tau=0.3, beta=0.5, K=20, mode="jfb", lr_theta=lr_t,
                   lr_lambda=lr_l)
    th0 = tr.theta.copy()
    _, g, gl = tr.epoch(Y, Xs)
    big = np.abs(g) > 1e-4
    assert big.sum() > 0.5 * g.size
    np.testing.assert_allclose((tr.theta - th0)[big], -lr_t * np.sign(g[big]), rtol=1e-3)
    assert abs((tr.lam - 0.7) + lr_l * np.sign(gl)) < 1e-3 * lr_l
    frozen = T.Trainer(net, op, 0.7, tau=0.3, beta=0.5, K=20, mode="jfb", learn_lambda=False)
    frozen.epoch(Y, Xs)
    assert frozen.lam == 0.7
