"""Failure detection and resume of the solver:
  * a step size of 10 / L makes the iteration blow up; the first update whose
    operand is larger than 1e6 times the initial iterate stops the image with
    IDQ_ST_DIVERGED, at the same update index as the float64 oracle's own
    iterates give;
  * a solve of 40 updates equals one of 20 updates resumed from its last
    iterate and the iterate before it (x_prev_out -> x_prev), bit for bit, with
    and without graph replay."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import net_layers, to_gpu, to_np
from oracle import operators as O, regularizer as R, solver as S
from paper_2605_19705_amd import IDQ, _lib as L

pytestmark = pytest.mark.gpu


def _denoise():
    layers = net_layers("gray16", 0)
    xt, nz = synth.make_batch(1, 2, 1, 32, 32)
    y = xt + 25.0 / 255.0 * nz
    P = S.Problem(O.Operator("identity"), R.Net(layers), 1.0)
    L_ = S.power_iteration(P, y, y, synth.random_field(12345, y.shape), 30)
    return layers, y, P, L_


def test_divergence_stops_at_the_oracle_index():
    """tau = 10 / L: the iterates grow ~9x per update while the relative step
    stays near 9, so the test is on the norm: the first update whose operand
    x^{k-1} is larger than 1e6 ||x^0|| stops the image, at the index the
    oracle's own iterates give."""
    print("divergence: tau = 10 / L, 2x1x32x32 f64", flush=True)
    layers, y, P, L_ = _denoise()
    tau = 10.0 / L_
    n0 = np.linalg.norm(y.reshape(2, -1), axis=1)
    want = [None, None]
    for j in range(1, 30):
        with np.errstate(all="ignore"):
            xj, _ = S.ideq_solve(P, y, y, 0.5, tau, fixed_iters=j)
        nj = np.linalg.norm(xj.reshape(2, -1), axis=1)
        for i in range(2):
            if want[i] is None and nj[i] > 1e6 * n0[i]:
                want[i] = j + 1
        if all(w is not None for w in want):
            break
    assert all(w is not None for w in want)
    ctx = IDQ(layers, op_kind="identity", device=0)
    x, res = ctx.solve(to_gpu(y), beta=0.5, tau=tau, lam=1.0, tol=1e-4, max_iter=200,
                       conv_prec="f64")
    assert res.code == L.IDQ_E_DIVERGED
    assert np.all(res.status == L.IDQ_ST_DIVERGED)
    assert res.iters.tolist() == want, (res.iters, want)
    # with the test off the same run goes on to max_iter or a non-finite iterate
    _, res2 = ctx.solve(to_gpu(y), beta=0.5, tau=tau, lam=1.0, tol=1e-4, max_iter=60,
                        conv_prec="f64", diverge_ratio=0.0)
    assert np.all(res2.status != L.IDQ_ST_DIVERGED)
    ctx.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_resume_equals_uninterrupted(use_graph):
    print(f"resume 20 + 20 vs 40 updates, graph={use_graph}", flush=True)
    layers, y, P, L_ = _denoise()
    tau = 0.9 / L_
    ctx = IDQ(layers, op_kind="identity", device=0)
    yg = to_gpu(y)
    kw = dict(beta=0.5, tau=tau, lam=1.0, conv_prec="f64", use_graph=use_graph)
    x40, _ = ctx.solve(yg, fixed_iters=40, **kw)
    xp = torch.empty_like(yg)
    x20, _ = ctx.solve(yg, fixed_iters=20, x_prev_out=xp, **kw)
    xr, r = ctx.solve(yg, x0=x20, x_prev=xp, fixed_iters=20, **kw)
    assert torch.equal(xr, x40)
    # without x_prev the resumed run loses the first step's inertia
    xn, _ = ctx.solve(yg, x0=x20, fixed_iters=20, **kw)
    assert not torch.equal(xn, x40)
    x_or, _ = S.ideq_solve(P, y, y, 0.5, tau, fixed_iters=40)
    assert float(np.max(np.abs(to_np(xr) - x_or))) < 1e-10
    ctx.close()
