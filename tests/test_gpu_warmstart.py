"""Parity of the learned warm start x0 = y + W_phi(y) (forward, loss gradient,
Adam steps, solver initialisation) against the float64 oracle.

Sizes: 2 x 3 x 40 x 36 spans 3 x 3 conv tiles of 16 x 16 at full resolution
(ragged in both directions) and 2 x 2 ragged tiles at half resolution (20 x 18).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import warmstart as WS

from gpu_util import to_gpu, to_np

pytestmark = pytest.mark.gpu

# float32 path: every operand and accumulation is float32 (weight gradients
# accumulate in float64); through 9 convs the relative error stays ~1e-6.
TOL_F32 = 2e-5
# bf16 path: activations and weights round to 8 mantissa bits (2^-9 relative
# each), float32 accumulation.  Measured on MI355X: 7.8e-3 for the network
# output, 4.5e-3 .. 7.9e-3 for the layers' gradients; the bound is the 2e-2
# relative tolerance of bf16 results.
TOL_BF16 = 2e-2


def _layers(seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for ci, co in synth.warmstart_channels():
        out.append((rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2 / (9 * ci)),
                    0.05 * rng.standard_normal(co)))
    return out


def _pair(n=2, h=40, w=36):
    xt, nz = synth.make_batch(11, n, 3, h, w)
    return xt + 0.1 * nz, xt


def _flat(pairs):
    return np.concatenate([np.concatenate([a.ravel(), b.ravel()]) for a, b in pairs])


def _ws(layers):
    from paper_2605_19705_amd import WarmStart
    return WarmStart(layers, device=0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_params_roundtrip_is_float32_master():
    layers = _layers()
    ws = _ws(layers)
    p = ws.get_params()
    flat = _flat(layers)
    assert p.shape == flat.shape
    assert np.array_equal(p, flat.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("prec,tol", [("f32", TOL_F32), ("bf16", TOL_BF16)])
def test_forward_matches_oracle(prec, tol):
    print(f"warm-start forward {prec} 2x3x40x36", flush=True)
    layers = _layers()
    y, _ = _pair()
    # the oracle runs on the float32-rounded weights and inputs the device sees
    l32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
           for W, b in layers]
    y32 = y.astype(np.float32).astype(np.float64)
    ref, _ = WS.forward(l32, y32)
    ws = _ws(layers)
    x0 = to_np(ws.forward(to_gpu(y, torch.float32), prec=prec))
    assert np.all(np.isfinite(x0))
    # compare the network output W_phi(y) = x0 - y
    err = _rel(x0 - y32, ref - y32)
    print(f"warm-start forward {prec}: relative error of W_phi(y) {err:.3e}", flush=True)
    assert err < tol, (prec, err)


@pytest.mark.parametrize("prec,tol", [("f32", TOL_F32 * 5), ("bf16", TOL_BF16)])
def test_loss_gradient_matches_oracle(prec, tol):
    print(f"warm-start gradient {prec} 2x3x40x36", flush=True)
    layers = _layers()
    y, t = _pair()
    l32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
           for W, b in layers]
    y32 = y.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    loss_ref, grads = WS.mse_loss_grad(l32, y32, t32)
    ws = _ws(layers)
    loss, g = ws.grad(to_gpu(y, torch.float32), to_gpu(t, torch.float32), prec=prec)
    g = to_np(g)
    assert abs(loss - loss_ref) < tol * loss_ref, (loss, loss_ref)
    off = 0
    for l, (dW, db) in enumerate(grads):
        gw = g[off:off + dW.size]
        gb = g[off + dW.size:off + dW.size + db.size]
        off += dW.size + db.size
        print(f"warm-start gradient {prec} layer {l}: W {_rel(gw, dW.ravel()):.3e} "
              f"b {_rel(gb, db.ravel()):.3e}", flush=True)
        assert _rel(gw, dW.ravel()) < tol, (prec, l, "W", _rel(gw, dW.ravel()))
        assert _rel(gb, db.ravel()) < tol, (prec, l, "b", _rel(gb, db.ravel()))
    assert off == g.size


def test_adam_step_matches_oracle():
    """First Adam step from zero moments: each parameter moves by -lr * g / (|g| + eps)
    (bias corrections cancel); compared where the oracle gradient is not tiny."""
    print("warm-start Adam step f32", flush=True)
    layers = _layers()
    y, t = _pair()
    l32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
           for W, b in layers]
    loss_ref, grads = WS.mse_loss_grad(l32, y.astype(np.float32).astype(np.float64),
                                       t.astype(np.float32).astype(np.float64))
    gref = _flat(grads)
    p0 = _flat(l32)
    lr = 1e-3
    p1_ref = WS.Adam(p0.size, lr=lr).step(p0, gref)
    ws = _ws(layers)
    loss = ws.train_step(to_gpu(y, torch.float32), to_gpu(t, torch.float32), lr, prec="f32")
    assert abs(loss - loss_ref) < 1e-4 * loss_ref
    p1 = ws.get_params()
    big = np.abs(gref) > 1e-2 * np.sqrt(np.mean(gref ** 2))
    assert big.mean() > 0.5
    step = p1 - p0
    np.testing.assert_allclose(step[big], (p1_ref - p0)[big], rtol=1e-3, atol=1e-7)
    assert np.all(np.abs(step) <= lr * 1.001 + 1e-7)


def _unflat(flat, like):
    out, off = [], 0
    for W, b in like:
        out.append((flat[off:off + W.size].reshape(W.shape),
                    flat[off + W.size:off + W.size + b.size]))
        off += W.size + b.size
    assert off == flat.size
    return out


def test_three_adam_steps_match_oracle():
    """Three float32 Adam steps against the oracle's own three steps, each taken
    at the oracle's own iterate.  From the second step on the bias corrections
    no longer cancel, and at lr 1e-3 most gradients change sign after the first
    step, so the moments mix values of both signs.  Compared where every oracle
    gradient of the three is above 0.1 rms: there a float32 gradient error e
    moves a step by about lr * e / |g|, and the tolerance 2e-3 * lr covers
    three steps at e up to 2e-5 rms (float32 gradients are near 1e-6)."""
    print("warm-start Adam, three f32 steps", flush=True)
    layers = _layers()
    y, t = _pair()
    l32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
           for W, b in layers]
    y32 = y.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    p0 = _flat(l32)
    lr = 1e-3
    opt = WS.Adam(p0.size, lr=lr)
    p_ref, gs = p0, []
    for _ in range(3):
        _, grads = WS.mse_loss_grad(_unflat(p_ref, l32), y32, t32)
        gs.append(_flat(grads))
        p_ref = opt.step(p_ref, gs[-1])
    ws = _ws(layers)
    yg, tg = to_gpu(y, torch.float32), to_gpu(t, torch.float32)
    for _ in range(3):
        ws.train_step(yg, tg, lr, prec="f32")
    p3 = ws.get_params()
    keep = np.all([np.abs(g) > 0.1 * np.sqrt(np.mean(g ** 2)) for g in gs], axis=0)
    assert keep.mean() > 0.2
    np.testing.assert_allclose((p3 - p0)[keep], (p_ref - p0)[keep], rtol=1e-3, atol=2e-3 * lr)


def test_training_lowers_the_loss():
    print("warm-start training, 30 bf16 Adam steps on 4x3x64x64", flush=True)
    xt, nz = synth.make_batch(12, 4, 3, 64, 64)
    y = to_gpu(xt + 0.1 * nz, torch.float32)
    t = to_gpu(xt, torch.float32)
    ws = _ws(_layers())
    losses = [ws.train_step(y, t, 2e-3, prec="bf16") for _ in range(30)]
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], losses


def test_solver_warm_start_equals_explicit_x0():
    """init="warmstart" runs the network inside idq_solve; passing the same
    network output as x0 must give the identical solve."""
    print("solve with warm-start init vs explicit x0, 2x3x32x32", flush=True)
    from paper_2605_19705_amd import IDQ
    layers = synth.he_normal_net(synth.net_channels("rgb64"), 0)
    taps = synth.gaussian_taps(9, 1.6)
    xt, nz = synth.make_batch(13, 2, 3, 32, 32)
    from oracle import operators as O
    y = to_gpu(O.Operator("blur", taps).A(xt) + 0.01 * nz, torch.float32)
    ctx = IDQ(layers, op_kind="blur", taps=taps, device=0)
    ws = _ws(_layers())
    kw = dict(beta=0.5, tau=0.17, lam=1.0, tol=1e-4, max_iter=300, conv_prec="f32")
    xa, ra = ctx.solve(y, init="warmstart", ws=ws, ws_prec="bf16", **kw)
    x0 = ws.forward(y, prec="bf16")
    xb, rb = ctx.solve(y, x0=x0, **kw)
    assert np.array_equal(ra.iters, rb.iters)
    assert np.array_equal(to_np(xa), to_np(xb))


# ---- the trained network shipped with the package --------------------------------
import os  # noqa: E402
import time  # noqa: E402

from gpu_util import rel_err  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2605_19705_amd", "weights", "warmstart_deblur.npy")


def _trained():
    assert os.path.exists(WEIGHTS), "trained warm-start weights missing from the package"
    from paper_2605_19705_amd import WarmStart
    return WarmStart(np.load(WEIGHTS).astype(np.float64), device=0)


def _deblur(cfg_id, n, size):
    from paper_2605_19705_amd import IDQ
    from oracle import operators as O
    layers = synth.he_normal_net(synth.net_channels("rgb64"), 0)
    taps = synth.gaussian_taps(9, 1.6)
    xt, nz = synth.make_batch(cfg_id, n, 3, size, size)
    y = O.Operator("blur", taps).A(xt) + 0.01 * nz
    return layers, taps, y, IDQ(layers, op_kind="blur", taps=taps, device=0)


def test_trained_warm_start_reaches_the_oracle_fixed_point_from_y():
    """A solve started from the trained warm start lands on the fixed point the
    oracle reaches from x0 = y (held-out image, 1 x 3 x 48 x 48)."""
    print("trained warm start vs oracle fixed point from y, 1x3x48x48", flush=True)
    from oracle import operators as O, regularizer as R, solver as S
    layers, taps, y, ctx = _deblur(5, 1, 48)
    P = S.Problem(O.Operator("blur", taps), R.Net(layers), 1.0)
    tau = 0.9 / S.power_iteration(P, y, y, synth.random_field(12345, y.shape), 30)
    x_or, info = S.ideq_solve(P, y, y, 0.5, tau, tol=1e-6, max_iter=3000)
    assert np.all(info["status"] == S.CONVERGED)
    ws = _trained()
    yg = to_gpu(y, torch.float32)
    kw = dict(beta=0.5, tau=tau, lam=1.0, max_iter=3000, init="warmstart", ws=ws, ws_prec="bf16")
    xbf, res = ctx.solve(yg, tol=1e-4, conv_prec="bf16", **kw)
    assert np.all(res.status == 0)
    assert rel_err(to_np(xbf), x_or) < 2e-2
    x32, res32 = ctx.solve(yg, tol=1e-6, conv_prec="f32", **kw)
    assert np.all(res32.status == 0)
    assert np.max(np.abs(to_np(x32) - x_or)) < 1e-4


def test_trained_warm_start_saves_iterations_at_512():
    """Held-out batch of 4 x 3 x 512 x 512: the headline solve (bf16 phase + fp32
    refinement to rel 1e-4) needs fewer iterations from the trained warm start than
    from y or from zero, and ends at the same fixed point."""
    print("trained warm start vs y / zero init, 4x3x512x512", flush=True)
    layers, taps, y, ctx = _deblur(5, 4, 512)
    yg = to_gpu(y, torch.float32)
    v0 = to_gpu(synth.random_field(12345, y.shape), torch.float32)
    tau = 0.9 / ctx.lipschitz(yg, yg, v0, lam=1.0, iters=30, conv_prec="f32")
    ws = _trained()
    kw = dict(beta=0.5, tau=tau, lam=1.0, tol=1e-4, max_iter=3000, conv_prec="bf16")
    out = {}
    for init in ("y", "zero", "warmstart"):
        extra = dict(ws=ws, ws_prec="bf16") if init == "warmstart" else {}
        ctx.solve(yg, init=init, **kw, **extra)        # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, res = ctx.solve(yg, init=init, **kw, **extra)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert np.all(res.status == 0), init
        out[init] = (to_np(x), res, dt)
        print(f"  init={init}: iterations {res.iters.tolist()} (bf16 {res.iters_low.tolist()}), "
              f"{4 / dt:.1f} images/s", flush=True)
    it = {k: float(np.mean(v[1].iters)) for k, v in out.items()}
    assert it["warmstart"] < it["y"] and it["warmstart"] < it["zero"], it
    assert rel_err(out["warmstart"][0], out["y"][0]) < 2e-2
