"""GPU parity of the fixed-point backward (App. D.1) against the float64 oracle,
in the training step's own arithmetic (float32) and through the autograd
wrapper.

The problem is the standalone 3 x 8 x 8 deblurring crop: the 5-layer 64-channel
network, the 9 x 9 circular blur (its taps wrap onto themselves on 8 x 8),
noise 0.01.  The oracle's fixed point is solved to rel 1e-14; the implicit
adjoint u* = (tau H_F)^{-1} v comes from the oracle's dense Hessian.  On this
crop tau H_F has eigenvalues in [0.038, 0.71], so float32 errors are amplified
at most ~19 times.

Tolerances (relative to the largest entry of the reference):
* float32 JFB at the oracle's fixed point: 1e-4 (float32 arithmetic, no solve);
* float32 implicit with adjoint_tol 1e-6: the adjoint's stopping error is about
  1e-6 / 0.04 ~ 2.5e-5 relative, so 1e-4;
* float64 through IDQSolve: 1e-7 (as the float64 crop backward);
* float32 through IDQSolve, forward solved to rel 1e-6: that iterate lies
  ~1.2e-5 (relative) from the fixed point, which the gradients inherit, so 1e-3.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import operators as O, regularizer as R, solver as S, backward as B

from gpu_util import to_gpu, to_np, net_layers

pytestmark = pytest.mark.gpu


def _crop_problem():
    layers = net_layers("rgb64", 0)
    taps = synth.gaussian_taps(9, 1.6)
    op = O.Operator("blur", taps)
    xt, nz = synth.make_batch(4, 1, 3, 8, 8)
    y = op.A(xt) + 0.01 * nz
    P = S.Problem(op, R.Net(layers), 1.0)
    tau = 0.9 / S.power_iteration(P, y, y, synth.random_field(12345, y.shape), 30)
    xbar, _ = S.ideq_solve(P, y, y, 0.5, tau, tol=1e-14, max_iter=20000)
    return layers, taps, xt, y, P, tau, xbar


def _ctx(layers, taps):
    from paper_2605_19705_amd import IDQ
    return IDQ(layers, op_kind="blur", taps=taps, device=0)


def _dense_adjoint(P, xbar, y, v, tau):
    H = B.dense_hessian(P, xbar, y)
    return np.linalg.solve(tau * 0.5 * (H + H.T), v.ravel()).reshape(v.shape)


def _flat(t):
    return to_np(t.reshape(1, 1, 1, -1)).ravel()


def test_backward_f32_on_crop():
    print("float32 JFB and implicit backward on the 3x8x8 crop vs the oracle", flush=True)
    layers, taps, xt, y, P, tau, xbar = _crop_problem()
    v = 2.0 * (xbar - xt) / xbar.size
    ctx = _ctx(layers, taps)
    f32 = lambda a: to_gpu(a, torch.float32)  # noqa: E731
    # JFB: u = v
    ref_th, ref_lam = B.theta_grad(P, xbar, y, v, tau)
    dth, dlam, _ = ctx.backward(f32(xbar), f32(y), f32(v), tau, 1.0, mode="jfb")
    assert dth.dtype == torch.float32
    assert np.max(np.abs(_flat(dth) - ref_th)) < 1e-4 * np.max(np.abs(ref_th))
    assert abs(dlam - ref_lam) < 1e-4 * abs(ref_lam)
    # implicit: u* = (tau H)^{-1} v
    u = _dense_adjoint(P, xbar, y, v, tau)
    ref_th, ref_lam = B.theta_grad(P, xbar, y, u, tau)
    dth, dlam, (iters, rel) = ctx.backward(f32(xbar), f32(y), f32(v), tau, 1.0, mode="implicit",
                                           adjoint_max_iter=20000, adjoint_tol=1e-6,
                                           adjoint_beta=0.5)
    assert rel < 1e-6 and 0 < iters < 20000
    assert np.max(np.abs(_flat(dth) - ref_th)) < 1e-4 * np.max(np.abs(ref_th))
    assert abs(dlam - ref_lam) < 1e-4 * abs(ref_lam)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_idqsolve_autograd_end_to_end(dtype):
    """x = IDQSolve.apply(y, theta, lam, ...); loss = mean((x - x_true)^2);
    loss.backward() fills theta.grad and lam.grad with the implicit gradient."""
    print(f"IDQSolve.apply + loss.backward() on the 3x8x8 crop, {dtype}", flush=True)
    from paper_2605_19705_amd import IDQSolve, pack_layers
    layers, taps, xt, y, P, tau, xbar = _crop_problem()
    ctx = _ctx(layers, taps)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    theta = torch.tensor(pack_layers(layers), dtype=torch.float64, requires_grad=True)
    lam = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    if dtype == "f64":
        skw = dict(beta=0.5, tau=tau, tol=1e-13, max_iter=20000, conv_prec="f64")
        bkw = dict(mode="implicit", adjoint_max_iter=100000, adjoint_tol=1e-13, adjoint_beta=0.5)
        tol = 1e-7
    else:
        skw = dict(beta=0.5, tau=tau, tol=1e-6, max_iter=20000, conv_prec="f32")
        bkw = dict(mode="implicit", adjoint_max_iter=20000, adjoint_tol=1e-6, adjoint_beta=0.5)
        tol = 1e-3
    yg = to_gpu(y, tdt)
    xtg = to_gpu(xt, tdt)
    x = IDQSolve.apply(yg, theta, lam, ctx, skw, bkw)
    loss = ((x - xtg) ** 2).mean()
    loss.backward()
    # oracle: v = dloss/dxbar at its own fixed point, u* by the dense solve
    v = 2.0 * (xbar - xt) / xbar.size
    u = _dense_adjoint(P, xbar, y, v, tau)
    ref_th, ref_lam = B.theta_grad(P, xbar, y, u, tau)
    assert theta.grad.dtype == torch.float64 and theta.grad.shape == theta.shape
    g = theta.grad.numpy()
    assert np.max(np.abs(g - ref_th)) < tol * np.max(np.abs(ref_th))
    assert abs(float(lam.grad) - ref_lam) < tol * abs(ref_lam)
    assert np.max(np.abs(to_np(x) - xbar)) < (1e-10 if dtype == "f64" else 1e-4)


def test_idqsolve_refuses_a_point_that_is_not_a_fixed_point():
    print("IDQSolve forward raises when an image stops on max_iter", flush=True)
    from paper_2605_19705_amd import IDQSolve, pack_layers
    from paper_2605_19705_amd._lib import IDQError
    layers, taps, xt, y, P, tau, xbar = _crop_problem()
    ctx = _ctx(layers, taps)
    theta = torch.tensor(pack_layers(layers), dtype=torch.float64, requires_grad=True)
    lam = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    with pytest.raises(IDQError):
        IDQSolve.apply(to_gpu(y), theta, lam, ctx,
                       dict(beta=0.5, tau=tau, tol=1e-14, max_iter=3, conv_prec="f64"),
                       dict(mode="jfb"))
    # a fixed iteration budget (the paper's training setting) is accepted
    x = IDQSolve.apply(to_gpu(y), theta, lam, ctx,
                       dict(beta=0.5, tau=tau, fixed_iters=5, conv_prec="f64"), dict(mode="jfb"))
    x.sum().backward()
    assert torch.isfinite(theta.grad).all()
