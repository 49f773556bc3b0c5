"""Pins for oracle.regularizer: central differences of g, grad g and the
parameter derivatives, Hessian symmetry, the per-channel reading, and the
linear-network special case against a dense matrix built with torch CPU."""
import numpy as np
import pytest
import torch

import synth
from oracle import regularizer as R


def small_net(chans=(3, 8, 8, 3), seed=0, act="softplus"):
    return R.Net(synth.he_normal_net(list(chans), seed, bias_seed=seed + 100), act)


def test_grad_by_central_differences(rng):
    net = small_net()
    x = rng.uniform(0, 1, (2, 3, 7, 6))
    g = net.grad(x)
    for _ in range(3):
        w = rng.standard_normal(x.shape)
        eps = 1e-5
        fd = (net.g(x + eps * w) - net.g(x - eps * w)) / (2 * eps)
        np.testing.assert_allclose(np.sum(g * w, axis=(1, 2, 3)), fd, rtol=1e-7)


def test_hvp_by_central_differences_and_symmetry(rng):
    net = small_net()
    x = rng.uniform(0, 1, (1, 3, 6, 7))
    u = rng.standard_normal(x.shape)
    v = rng.standard_normal(x.shape)
    eps = 1e-5
    fd = (net.grad(x + eps * u) - net.grad(x - eps * u)) / (2 * eps)
    hu = net.hvp(x, u)
    np.testing.assert_allclose(hu, fd, atol=2e-8 * np.max(np.abs(hu)))
    assert abs(np.sum(hu * v) - np.sum(u * net.hvp(x, v))) < 1e-11 * np.sum(np.abs(hu * v))


def test_param_grad_by_central_differences(rng):
    net = small_net()
    x = rng.uniform(0, 1, (2, 3, 5, 6))
    p = net.pack()
    d = rng.standard_normal(p.size)
    d /= np.linalg.norm(d)
    eps = 1e-4
    fd = (net.with_params(p + eps * d).g(x).sum() - net.with_params(p - eps * d).g(x).sum()) / (2 * eps)
    an = np.dot(R.pack_grads(net.param_grad(x)), d)
    assert abs(fd - an) < 1e-7 * abs(an)


def test_mixed_grad_by_central_differences(rng):
    net = small_net()
    x = rng.uniform(0, 1, (2, 3, 5, 6))
    u = rng.standard_normal(x.shape)
    p = net.pack()
    an = R.pack_grads(net.mixed_grad(x, u))
    for _ in range(2):
        d = rng.standard_normal(p.size)
        d /= np.linalg.norm(d)
        eps = 1e-4
        fp = np.sum(u * net.with_params(p + eps * d).grad(x))
        fm = np.sum(u * net.with_params(p - eps * d).grad(x))
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - np.dot(an, d)) < 1e-7 * abs(fd)


def test_per_channel_application(rng):
    net = R.Net(synth.he_normal_net(synth.net_channels("gray16"), 0))
    x = rng.uniform(0, 1, (2, 3, 6, 5))
    g = net.grad(x)
    for c in range(3):
        np.testing.assert_allclose(g[:, c:c + 1], net.grad(x[:, c:c + 1]), atol=1e-14)


def dense_linear_net(layers, c, h, w):
    """N(x) = W_eff x + c0 for an identity-activation net, via torch conv2d."""
    d = c * h * w

    def Nt(t):
        for W, b in layers:
            t = torch.nn.functional.conv2d(t, torch.from_numpy(W), torch.from_numpy(b), padding=1)
        return t

    with torch.no_grad():
        c0 = Nt(torch.zeros(1, c, h, w, dtype=torch.float64)).numpy().ravel()
        basis = torch.eye(d, dtype=torch.float64).reshape(d, c, h, w)
        cols = Nt(basis).numpy().reshape(d, d) - c0[None, :]
    return cols.T, c0


def test_linear_network_gradient_is_quadratic_form(rng):
    layers = synth.he_normal_net([1, 4, 4, 1], 3, bias_seed=7)
    net = R.Net(layers, act="identity")
    h, w = 5, 6
    Weff, c0 = dense_linear_net(layers, 1, h, w)
    M = np.eye(h * w) - Weff
    x = rng.standard_normal((1, 1, h, w))
    ref = M.T @ (M @ x.ravel() - c0)
    np.testing.assert_allclose(net.grad(x).ravel(), ref, atol=1e-12)
    u = rng.standard_normal(x.shape)
    np.testing.assert_allclose(net.hvp(x, u).ravel(), M.T @ M @ u.ravel(), atol=1e-12)
