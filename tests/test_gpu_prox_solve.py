"""GPU parity of whole solves on the inpainting, MRI and Rician workloads and
of the proximal i-DEQ-P iteration (App. B, Alg. 2) against the oracle:
  * trajectory parity: same x^0, same tau, K fixed updates, float64 at 1e-10
    max-abs and float32 at 1e-4 (the protocol of the Alg. 1 workloads);
  * fixed-point parity of a bf16 -> float32 solve to the oracle's fixed point;
  * the options the proximal form refuses.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import net_layers, rel_err, to_gpu, to_np
from oracle import operators as O, regularizer as R, solver as S
from paper_2605_19705_amd import IDQ, _lib as L

pytestmark = pytest.mark.gpu


def workload(kind, n, c, h, w, seed):
    """(oracle operator, IDQ kwargs, x_true, y, net name)."""
    xt, nz = synth.make_batch(40 + seed, n, c, h, w)
    rng = np.random.default_rng(seed)
    if kind == "inpaint":
        m = synth.pixel_mask(seed, h, w, 0.5)
        op = O.Operator("inpaint", mask=m)
        y = op.A(xt) + 5.0 / 255.0 * nz
        return op, dict(op_kind="inpaint", mask=m), xt, y
    if kind == "mri":
        m = synth.cartesian_mask(seed, h, w, accel=8)
        op = O.Operator("mri", mask=m)
        nzi = rng.standard_normal(xt.shape)
        y = op.A(xt) + (1.0 / 255.0) * op.mask * (nz + 1j * nzi)
        return op, dict(op_kind="mri", mask=m), xt, y
    if kind == "rician":
        s = 25.5 / 255.0
        nzi = rng.standard_normal(xt.shape)
        y = np.sqrt((xt + s * nz) ** 2 + (s * nzi) ** 2)
        return O.Operator("rician", sigma=s), dict(op_kind="rician", sigma=s), xt, y
    if kind == "blur":
        k = synth.gaussian_taps(9, 1.6)
        op = O.Operator("blur", k)
        return op, dict(op_kind="blur", taps=k), xt, op.A(xt) + 0.01 * nz
    raise ValueError(kind)


def gpu_y(y, dt):
    if np.iscomplexobj(y):
        cd = torch.complex128 if dt == torch.float64 else torch.complex64
        return torch.from_numpy(np.ascontiguousarray(y)).to(device="cuda", dtype=cd)
    return to_gpu(y, dt)


def x_start(op, y):
    """x^0 of a solve started 'from y': A^T y for MRI (y lives in k-space)."""
    return op.vjp(None, y) if op.kind == "mri" else y


CASES = [  # (kind, proximal, net, shape, lambda)
    ("inpaint", True, "gray16", (2, 1, 32, 32), 1.0),
    ("inpaint", False, "gray16", (1, 3, 16, 32), 1.0),
    ("mri", True, "gray16", (2, 1, 32, 32), 0.5),
    ("mri", False, "gray16", (1, 1, 64, 32), 0.5),
    ("rician", False, "gray16", (2, 3, 16, 16), 0.05),
    ("blur", True, "gray16", (1, 3, 32, 16), 1.0),
]


@pytest.mark.parametrize("kind,proximal,net,shape,lam", CASES)
def test_trajectory_parity(kind, proximal, net, shape, lam):
    print(f"prox-solve: {kind} proximal={proximal} {shape}", flush=True)
    op, kw, xt, y = workload(kind, *shape, seed=1)
    layers = net_layers(net, 0, bias_seed=4)
    P = S.Problem(op, R.Net(layers), lam)
    x0 = x_start(op, y)
    tau = 0.9 / S.power_iteration(P, x0, y, synth.random_field(12345, x0.shape), 30)
    K = 40
    x_or, info = S.ideq_solve(P, y, x0, 0.5, tau, proximal=proximal, fixed_iters=K)
    ctx = IDQ(layers, **kw, device=0)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        dt = torch.float64 if prec == "f64" else torch.float32
        xg, res = ctx.solve(gpu_y(y, dt), x0=to_gpu(x0, dt), beta=0.5, tau=tau, lam=lam,
                            fixed_iters=K, proximal=proximal, conv_prec=prec)
        err = float(np.max(np.abs(to_np(xg) - x_or)))
        assert err < tol, (prec, err)
        assert np.all(res.iters == K) and np.all(res.status == L.IDQ_ST_FIXED)
    ctx.close()


@pytest.mark.parametrize("kind,proximal", [("inpaint", True), ("mri", True), ("rician", False)])
def test_bf16_then_f32_reaches_the_oracle_fixed_point(kind, proximal):
    print(f"prox-solve fixed point: {kind}", flush=True)
    shape = (1, 3, 32, 32) if kind == "rician" else (1, 1, 32, 32)
    op, kw, xt, y = workload(kind, *shape, seed=2)
    layers = net_layers("gray16", 0)
    lam = 0.05 if kind == "rician" else 1.0
    P = S.Problem(op, R.Net(layers), lam)
    x0 = x_start(op, y)
    tau = 0.9 / S.power_iteration(P, x0, y, synth.random_field(12345, x0.shape), 30)
    x_or, info = S.ideq_solve(P, y, x0, 0.5, tau, proximal=proximal, tol=1e-9, max_iter=3000)
    assert info["status"][0] == S.CONVERGED
    ctx = IDQ(layers, **kw, device=0)
    xg, res = ctx.solve(gpu_y(y, torch.float32), x0=to_gpu(x0, torch.float32), beta=0.5,
                        tau=tau, lam=lam, tol=1e-6, max_iter=3000, proximal=proximal,
                        conv_prec="bf16", refine_prec="f32", poll_every=4)
    assert np.all(res.status == L.IDQ_ST_CONVERGED)
    assert res.iters_low[0] > 0
    assert rel_err(to_np(xg), x_or) < 2e-2
    ctx.close()


def test_mri_init_y_is_the_zero_filled_image():
    op, kw, xt, y = workload("mri", 1, 1, 16, 16, seed=3)
    layers = net_layers("gray16", 0)
    ctx = IDQ(layers, **kw, device=0)
    yg = gpu_y(y, torch.float64)
    xg, _ = ctx.solve(yg, beta=0.5, tau=0.5, lam=1.0, fixed_iters=1, init="y")
    P = S.Problem(op, R.Net(layers), 1.0)
    x_or, _ = S.ideq_solve(P, y, op.vjp(None, y), 0.5, 0.5, fixed_iters=1)
    assert float(np.max(np.abs(to_np(xg) - x_or))) < 1e-12
    ctx.close()


def test_proximal_refusals():
    layers = net_layers("gray16", 0)
    y = torch.zeros((1, 1, 8, 8), dtype=torch.float64, device="cuda")
    for kw in (dict(op_kind="rician", sigma=0.1),
               dict(op_kind="tanh_blur", taps=synth.uniform_taps(3), gain=2.0)):
        ctx = IDQ(layers, **kw, device=0)
        with pytest.raises(L.IDQError) as e:
            ctx.solve(y, tau=0.5, fixed_iters=2, proximal=True)
        assert e.value.code == L.IDQ_E_UNSUPPORTED
        ctx.close()
    ctx = IDQ(layers, op_kind="identity", device=0)
    with pytest.raises(L.IDQError) as e:
        ctx.solve(y, tau=0.5, fixed_iters=2, proximal=True, grad_at="current")
    assert e.value.code == L.IDQ_E_UNSUPPORTED
    ctx.close()
