"""Pins for oracle.warmstart: central differences of the MSE loss through the
encoder-decoder, the pooling/upsampling adjoint pairs, and Adam's steps by
closed forms (first step, a constant gradient, a gradient then a zero one)."""
import numpy as np

import synth
from oracle import warmstart as WS


def ws_layers(seed=1):
    out = []
    rng = np.random.default_rng(seed)
    for ci, co in synth.warmstart_channels():
        out.append((rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2 / (9 * ci)),
                    0.05 * rng.standard_normal(co)))
    return out


def test_pool_upsample_adjoints(rng):
    x = rng.standard_normal((2, 3, 6, 8))
    g = rng.standard_normal((2, 3, 3, 4))
    assert abs(np.sum(WS.avgpool2(x) * g) - np.sum(x * WS.avgpool2_adjoint(g))) < 1e-12
    assert abs(np.sum(WS.upsample2(g) * x) - np.sum(g * WS.upsample2_adjoint(x))) < 1e-12
    np.testing.assert_allclose(WS.avgpool2(np.ones((1, 1, 4, 4))), np.ones((1, 1, 2, 2)))


def test_loss_gradient_by_central_differences(rng):
    layers = ws_layers()
    y = rng.uniform(0, 1, (2, 3, 8, 6))
    t = rng.uniform(0, 1, (2, 3, 8, 6))
    loss, grads = WS.mse_loss_grad(layers, y, t)
    flat = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])
    gflat = np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in grads])

    def unflat(f):
        out, o = [], 0
        for W, b in layers:
            out.append((f[o:o + W.size].reshape(W.shape), f[o + W.size:o + W.size + b.size]))
            o += W.size + b.size
        return out

    for _ in range(3):
        d = rng.standard_normal(flat.size)
        eps = 1e-6
        lp, _ = WS.mse_loss_grad(unflat(flat + eps * d), y, t)
        lm, _ = WS.mse_loss_grad(unflat(flat - eps * d), y, t)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - np.dot(gflat, d)) < 1e-6 * abs(fd)


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    opt = WS.Adam(3, lr=1e-2)
    p1 = opt.step(p, g)
    np.testing.assert_allclose(p1, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_constant_gradient_moves_lr_per_step():
    # with g fixed, the bias-corrected moments are exactly g and g^2 at every
    # step t, so each step is lr * g / (|g| + eps) whatever t is
    g = np.array([0.7, -1.5, 2e-4, -3e-2])
    p0 = np.array([1.0, -2.0, 0.5, 0.0])
    opt = WS.Adam(4, lr=3e-3)
    p = p0
    for _ in range(50):
        p = opt.step(p, g)
    np.testing.assert_allclose(p, p0 - 50 * 3e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_adam_zero_gradient_after_one_step_uses_decayed_moments():
    # m_2 = b1 (1 - b1) g and v_2 = b2 (1 - b2) g^2, so after bias correction
    # mhat = b1 g / (1 + b1) and vhat = b2 g^2 / (1 + b2)
    b1, b2, lr, eps = 0.9, 0.999, 1e-2, 1e-8
    g = np.array([0.4, -3.0, 1e-5])
    opt = WS.Adam(3, lr=lr, b1=b1, b2=b2, eps=eps)
    p1 = opt.step(np.zeros(3), g)
    p2 = opt.step(p1, np.zeros(3))
    want = lr * (b1 / (1 + b1)) * g / (np.sqrt(b2 / (1 + b2)) * np.abs(g) + eps)
    np.testing.assert_allclose(p1 - p2, want, rtol=1e-10)
