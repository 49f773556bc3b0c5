"""GPU parity of the training loop (Alg. 1 epochs; Alg. 2 for i-DEQ-P) with
the oracle's: three epochs (forward K updates, JFB or implicit gradient
accumulated over the pairs in two passes, one Adam step on theta and lambda),
each compared after every epoch.

float64: every parameter to 1e-10 (gradients agree to rounding, Adam keeps
that).  float32: where every oracle gradient of the three epochs is above
0.1 rms (a float32 gradient error e moves a step by about lr e / |g|), to
rtol 1e-3 and 2e-3 lr, as for the warm start's Adam steps; lambda to 1e-3 lr.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import net_layers, to_gpu
from oracle import operators as O, regularizer as R, solver as S, training as T
from paper_2605_19705_amd import IDQ, Trainer

pytestmark = pytest.mark.gpu


def dataset(kind, N, c, h, w, seed=7):
    xt, nz = synth.make_batch(50 + seed, N, c, h, w)
    if kind == "blur":
        k = synth.gaussian_taps(5, 1.0)
        op = O.Operator("blur", k)
        return op, dict(op_kind="blur", taps=k), op.A(xt) + 0.01 * nz, xt
    if kind == "inpaint":
        m = synth.pixel_mask(seed, h, w, 0.5)
        op = O.Operator("inpaint", mask=m)
        return op, dict(op_kind="inpaint", mask=m), op.A(xt) + 0.02 * nz, xt
    if kind == "mri":
        m = synth.cartesian_mask(seed, h, w, accel=4)
        op = O.Operator("mri", mask=m)
        rng = np.random.default_rng(seed)
        y = op.A(xt) + 0.01 * op.mask * (nz + 1j * rng.standard_normal(xt.shape))
        return op, dict(op_kind="mri", mask=m), y, xt
    raise ValueError(kind)


def gpu_data(a, dt):
    if np.iscomplexobj(a):
        cd = torch.complex128 if dt == torch.float64 else torch.complex64
        return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=cd)
    return to_gpu(a, dt)


CASES = [  # kind, mode, proximal, averaging, shape (N, c, h, w)
    ("blur", "jfb", False, False, (4, 1, 16, 16)),
    ("blur", "implicit", False, True, (4, 1, 16, 16)),
    ("inpaint", "implicit", True, False, (4, 1, 16, 16)),
    ("mri", "jfb", True, False, (4, 1, 16, 16)),
]


@pytest.mark.parametrize("kind,mode,proximal,averaging,shape", CASES)
def test_three_epochs_match_the_oracle_f64(kind, mode, proximal, averaging, shape):
    print(f"training f64: {kind} {mode} proximal={proximal} averaging={averaging}", flush=True)
    op, kw, Y, Xs = dataset(kind, *shape)
    layers = net_layers("gray16", 0, bias_seed=3)
    lam0, tau, beta, K = 0.8, 0.2, 0.5, 30
    lr_t, lr_l = 2e-3, 1e-2
    ref = T.Trainer(R.Net(layers), op, lam0, tau=tau, beta=beta, K=K, mode=mode,
                    lr_theta=lr_t, lr_lambda=lr_l, averaging=averaging, proximal=proximal,
                    adjoint_iters=400, adjoint_tol=1e-12)
    ctx = IDQ(layers, **kw, device=0)
    tr = Trainer(ctx, lam0)
    Yg, Xg = gpu_data(Y, torch.float64), gpu_data(Xs, torch.float64)
    for ep in range(3):
        l_ref, _, _ = ref.epoch(Y, Xs, batch=2)
        l_gpu = tr.epoch(Yg, Xg, K=K, beta=beta, tau=tau, mode=mode, averaging=averaging,
                         proximal=proximal, lr_theta=lr_t, lr_lambda=lr_l,
                         adjoint_max_iter=400, adjoint_tol=1e-12, batch=2)
        th, lam = tr.params()
        assert abs(l_gpu - l_ref) < 1e-12 * max(1.0, l_ref), (ep, l_gpu, l_ref)
        np.testing.assert_allclose(th, ref.theta, rtol=0, atol=1e-10)
        assert abs(lam - ref.lam) < 1e-10, (ep, lam, ref.lam)
    tr.close()
    ctx.close()


def test_three_epochs_match_the_oracle_f32():
    print("training f32: blur jfb", flush=True)
    op, kw, Y, Xs = dataset("blur", 4, 3, 16, 16)
    layers = net_layers("rgb64", 0)
    l32 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
           for W, b in layers]
    Y32, X32 = (a.astype(np.float32).astype(np.float64) for a in (Y, Xs))
    lam0, tau, beta, K = 0.8, 0.1, 0.5, 20
    lr_t, lr_l = 1e-3, 1e-2
    ref = T.Trainer(R.Net(l32), op, lam0, tau=tau, beta=beta, K=K, mode="jfb", lr_theta=lr_t,
                    lr_lambda=lr_l)
    th0_ref = ref.theta.copy()
    gs = []
    for _ in range(3):
        _, g, _ = ref.epoch(Y32, X32, batch=2)
        gs.append(g)
    ctx = IDQ(layers, **kw, device=0)
    tr = Trainer(ctx, lam0)
    th0, _ = tr.params()
    Yg, Xg = to_gpu(Y, torch.float32), to_gpu(Xs, torch.float32)
    for _ in range(3):
        tr.epoch(Yg, Xg, K=K, beta=beta, tau=tau, mode="jfb", lr_theta=lr_t, lr_lambda=lr_l,
                 batch=2)
    th, lam = tr.params()
    keep = np.all([np.abs(g) > 0.1 * np.sqrt(np.mean(g ** 2)) for g in gs], axis=0)
    assert keep.mean() > 0.2
    np.testing.assert_allclose((th - th0)[keep], (ref.theta - th0_ref)[keep], rtol=1e-3,
                               atol=2e-3 * lr_t)
    assert abs(lam - ref.lam) < 3e-3 * lr_l, (lam, ref.lam)
    tr.close()
    ctx.close()


def test_training_lowers_the_loss():
    """Ten JFB epochs of Alg. 1 on 8 deblurring pairs of 1 x 32 x 32 (float32):
    the epoch loss falls (the oracle, run on the same data, falls from 0.38 to
    0.02 over 15 epochs)."""
    print("training: 10 f32 epochs on 8x1x32x32", flush=True)
    op, kw, Y, Xs = dataset("blur", 8, 1, 32, 32, seed=9)
    layers = net_layers("gray16", 0)
    P = S.Problem(op, R.Net(layers), 0.5)
    tau = 0.9 / S.power_iteration(P, Y[:1], Y[:1], synth.random_field(12345, Y[:1].shape), 30)
    ctx = IDQ(layers, **kw, device=0)
    tr = Trainer(ctx, 0.5)
    Yg, Xg = to_gpu(Y, torch.float32), to_gpu(Xs, torch.float32)
    losses = [tr.epoch(Yg, Xg, K=30, beta=0.5, tau=tau, mode="jfb", lr_theta=1e-3, lr_lambda=1e-2)
              for _ in range(10)]
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.2 * losses[0], losses
    tr.close()
    ctx.close()
