"""Pins for oracle.conv: an independent library (torch CPU conv2d), brute force
on a tiny input, the adjoint identity and exact linearity of the weight grad."""
import numpy as np
import pytest
import torch

from oracle import conv as C


def test_conv_matches_torch_conv2d(rng):
    x = rng.standard_normal((2, 5, 7, 9))
    W = rng.standard_normal((4, 5, 3, 3))
    b = rng.standard_normal(4)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(W),
                                     torch.from_numpy(b), padding=1).numpy()
    np.testing.assert_allclose(C.conv3x3(x, W, b), ref, rtol=0, atol=1e-12)


def test_conv_brute_force_tiny(rng):
    x = rng.standard_normal((1, 2, 3, 4))
    W = rng.standard_normal((3, 2, 3, 3))
    out = np.zeros((1, 3, 3, 4))
    for o in range(3):
        for i in range(3):
            for j in range(4):
                s = 0.0
                for c in range(2):
                    for dy in range(3):
                        for dx in range(3):
                            ii, jj = i + dy - 1, j + dx - 1
                            if 0 <= ii < 3 and 0 <= jj < 4:
                                s += W[o, c, dy, dx] * x[0, c, ii, jj]
                out[0, o, i, j] = s
    np.testing.assert_allclose(C.conv3x3(x, W), out, atol=1e-13)


def test_adjoint_dot(rng):
    x = rng.standard_normal((2, 3, 6, 5))
    d = rng.standard_normal((2, 4, 6, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    lhs = np.sum(C.conv3x3(x, W) * d)
    rhs = np.sum(x * C.conv3x3_adjoint(d, W))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_adjoint_matches_torch_transpose(rng):
    d = rng.standard_normal((1, 4, 6, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    ref = torch.nn.functional.conv_transpose2d(torch.from_numpy(d), torch.from_numpy(W),
                                               padding=1).numpy()
    np.testing.assert_allclose(C.conv3x3_adjoint(d, W), ref, atol=1e-12)


def test_wgrad_is_exact_derivative(rng):
    x = rng.standard_normal((2, 3, 5, 6))
    g = rng.standard_normal((2, 4, 5, 6))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    D, db_dir = rng.standard_normal(W.shape), rng.standard_normal(4)
    dW, db = C.conv3x3_wgrad(g, x)
    eps = 1e-3  # the map is linear in (W, b): central differences are exact
    fp = np.sum(g * C.conv3x3(x, W + eps * D, b + eps * db_dir))
    fm = np.sum(g * C.conv3x3(x, W - eps * D, b - eps * db_dir))
    fd = (fp - fm) / (2 * eps)
    assert abs(fd - (np.sum(dW * D) + np.sum(db * db_dir))) < 1e-9 * abs(fd)


def test_softplus_and_derivatives():
    t = np.array([-800.0, -30.0, -1.0, 0.0, 0.5, 30.0, 800.0])
    sp = C.softplus(t)
    assert np.all(np.isfinite(sp))
    np.testing.assert_allclose(sp[2:6], np.log1p(np.exp(t[2:6])), rtol=1e-14)
    assert sp[-1] == 800.0 and sp[0] == 0.0
    s, ds, d2s = C.activation("softplus")
    tt = np.linspace(-6, 6, 25)
    h = 1e-5
    np.testing.assert_allclose(ds(tt), (s(tt + h) - s(tt - h)) / (2 * h), atol=1e-9)
    np.testing.assert_allclose(d2s(tt), (ds(tt + h) - ds(tt - h)) / (2 * h), atol=1e-9)
