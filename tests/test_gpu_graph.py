"""HIP-graph replay of fixed-iteration solves: the steps replayed from the
graph must give bit-for-bit the iterates of the solve that launches every
kernel, for odd and even step counts, operators with Fourier and stencil
passes, and on repeated calls with other work and synchronisations between
them; and the float64 denoising solve (100 updates) must still match the
oracle to 1e-10."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import net_layers, to_gpu, to_np
from oracle import operators as O, regularizer as R, solver as S
from paper_2605_19705_amd import IDQ

pytestmark = pytest.mark.gpu


def test_denoising_100_updates_graph_equals_eager_and_oracle():
    print("graph: denoising 1x1x32x32 f64, 100 updates", flush=True)
    layers = net_layers("gray16", 0)
    xt, nz = synth.make_batch(1, 1, 1, 32, 32)
    y = xt + 25.0 / 255.0 * nz
    P = S.Problem(O.Operator("identity"), R.Net(layers), 1.0)
    tau = 0.9 / S.power_iteration(P, y, y, synth.random_field(12345, y.shape), 30)
    x_or, _ = S.ideq_solve(P, y, y, 0.5, tau, fixed_iters=100)
    ctx = IDQ(layers, op_kind="identity", device=0)
    yg = to_gpu(y)
    xe, re = ctx.solve(yg, beta=0.5, tau=tau, lam=1.0, fixed_iters=100, conv_prec="f64",
                       use_graph=False)
    for rep in range(3):
        xg, rg = ctx.solve(yg, beta=0.5, tau=tau, lam=1.0, fixed_iters=100, conv_prec="f64")
        assert torch.equal(xg, xe), rep
        assert np.array_equal(rg.iters, re.iters) and np.array_equal(rg.status, re.status)
        # other work on the device between the calls
        junk = torch.randn(1 << 20, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        del junk
    assert float(np.max(np.abs(to_np(xe) - x_or))) < 1e-10
    ctx.close()


@pytest.mark.parametrize("K", [3, 4, 17])
@pytest.mark.parametrize("kind", ["blur", "mri_prox", "inpaint_prox"])
def test_graph_equals_eager(kind, K):
    print(f"graph: {kind}, {K} updates", flush=True)
    n, c, h, w = 2, 1, 32, 32
    xt, nz = synth.make_batch(60, n, c, h, w)
    layers = net_layers("gray16", 0, bias_seed=2)
    if kind == "blur":
        kw = dict(op_kind="blur", taps=synth.gaussian_taps(9, 1.6))
        y = O.Operator("blur", kw["taps"]).A(xt) + 0.01 * nz
        yg, prox = to_gpu(y, torch.float32), False
    elif kind == "inpaint_prox":
        m = synth.pixel_mask(6, h, w)
        kw = dict(op_kind="inpaint", mask=m)
        yg, prox = to_gpu(O.Operator("inpaint", mask=m).A(xt) + 0.02 * nz, torch.float32), True
    else:
        m = synth.cartesian_mask(6, h, w, accel=4)
        kw = dict(op_kind="mri", mask=m)
        yk = O.Operator("mri", mask=m).A(xt)
        yg = torch.from_numpy(yk).to(device="cuda", dtype=torch.complex64)
        prox = True
    ctx = IDQ(layers, **kw, device=0)
    opts = dict(beta=0.5, tau=0.1, lam=1.0, fixed_iters=K, conv_prec="f32", proximal=prox)
    xe, _ = ctx.solve(yg, use_graph=False, **opts)
    for _ in range(2):
        xg, _ = ctx.solve(yg, **opts)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe)
    ctx.close()
