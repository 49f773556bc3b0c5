"""GPU property tests that need no oracle: images of a batch are independent,
so solving a batch must reproduce every image's single-image solve exactly
(same kernels, same per-image reductions), whatever mix of precision phases
the images are in and however many tiles each persistent workgroup walks;
invalid inputs are rejected with an error; the profiler's accounting."""
import numpy as np
import pytest
import torch

import synth
from oracle import operators as O

from gpu_util import to_gpu, to_np, net_layers

pytestmark = pytest.mark.gpu


def _ctx(layers, kind, taps):
    from paper_2605_19705_amd import IDQ
    return IDQ(layers, op_kind=kind, taps=taps, device=0)


def _deblur_batch(n, h, w):
    taps = synth.gaussian_taps(9, 1.6)
    op = O.Operator("blur", taps)
    xt, nz = synth.make_batch(2, n, 3, h, w)
    return taps, op.A(xt) + 0.01 * nz


def test_grad_reg_batch_equals_single_images_many_tiles():
    """2 x 3 x 256 x 256 is 512 tiles per pass: each workgroup of the
    persistent conv grid walks several tiles."""
    print("grad_reg bf16/f32 at 2x3x256x256 vs single images", flush=True)
    layers = net_layers("rgb64", 0)
    taps, y = _deblur_batch(2, 256, 256)
    ctx = _ctx(layers, "blur", taps)
    yb = to_gpu(y, torch.float32)
    for prec in ("f32", "bf16"):
        gb = to_np(ctx.grad_reg(yb, conv_prec=prec))
        for i in range(2):
            gi = to_np(ctx.grad_reg(yb[i:i + 1].contiguous(), conv_prec=prec))
            assert np.array_equal(gb[i:i + 1], gi), prec


def test_bf16_solve_batch_with_mixed_phases_equals_single_images():
    print("bf16 solve, 4 x 3 x 48 x 48, mixed phases", flush=True)
    layers = net_layers("rgb64", 0)
    taps, y = _deblur_batch(4, 48, 48)
    ctx = _ctx(layers, "blur", taps)
    yb = to_gpu(y, torch.float32)
    kw = dict(beta=0.5, tau=0.17, lam=1.0, tol=1e-4, max_iter=2000, conv_prec="bf16",
              switch_tol=1e-3, switch_patience=10)
    xb, rb = ctx.solve(yb, **kw)
    assert np.all(rb.status == 0)
    # the images leave the bf16 phase at different iterations
    assert len(set(rb.iters_low.tolist())) > 1
    for i in range(4):
        xi, ri = ctx.solve(yb[i:i + 1].contiguous(), **kw)
        assert ri.iters[0] == rb.iters[i] and ri.iters_low[0] == rb.iters_low[i]
        assert np.array_equal(to_np(xi), to_np(xb[i:i + 1]))


def test_profile_counts_pixels_and_launches():
    print("profiler accounting", flush=True)
    layers = net_layers("rgb64", 0)
    taps, y = _deblur_batch(2, 40, 56)
    ctx = _ctx(layers, "blur", taps)
    yb = to_gpu(y, torch.float32)
    ctx.profile(True)
    ctx.grad_reg(yb, conv_prec="bf16")
    ctx.grad_reg(yb, conv_prec="f32")
    prof = ctx.profile_read()
    ctx.profile(False)
    # 3 forward + 3 backward 64->64 passes per gradient, every pixel once
    assert prof["conv64_bf16"][1] == 6 and prof["conv64_f32"][1] == 6
    assert prof["conv64_bf16"][2] == 6 * 2 * 40 * 56
    assert prof["conv64_f32"][2] == 6 * 2 * 40 * 56
    assert prof["conv64_bf16"][0] > 0 and prof["conv_other"][1] == 8


def test_split_solve_batch_with_mixed_phases_equals_single_images():
    """bf16 -> split-bf16 -> float32 with polls every 3 steps: images leave the
    phases at different steps and wait for the float32 passes at different
    times, yet each reproduces its single-image solve bit for bit."""
    print("bf16 -> split -> f32 solve, 4 x 3 x 40 x 40, batch vs single images", flush=True)
    layers = net_layers("rgb64", 0)
    taps, y = _deblur_batch(4, 40, 40)
    ctx = _ctx(layers, "blur", taps)
    yb = to_gpu(y, torch.float32)
    kw = dict(beta=0.5, tau=0.17, lam=1.0, tol=1e-4, max_iter=2000, conv_prec="bf16",
              refine_prec="bf16x3", poll_every=3)
    xb, rb = ctx.solve(yb, **kw)
    assert np.all(rb.status == 0)
    assert np.all(rb.iters_mid > 0) and np.all(rb.iters > rb.iters_low + rb.iters_mid)
    print("  phase lengths (bf16, split, total):",
          list(zip(rb.iters_low.tolist(), rb.iters_mid.tolist(), rb.iters.tolist())), flush=True)
    for i in range(4):
        xi, ri = ctx.solve(yb[i:i + 1].contiguous(), **kw)
        assert (ri.iters[0], ri.iters_low[0], ri.iters_mid[0]) == \
            (rb.iters[i], rb.iters_low[i], rb.iters_mid[i])
        assert np.array_equal(to_np(xi), to_np(xb[i:i + 1]))


def test_invalid_inputs_are_rejected():
    """An empty batch, an empty image, channels the network does not take and a
    bad profiler sampling interval come back as library errors (IDQ_E_INVAL)."""
    import paper_2605_19705_amd._lib as L
    layers = net_layers("rgb64", 0)
    taps = synth.gaussian_taps(9, 1.6)
    ctx = _ctx(layers, "blur", taps)
    for shape in ((0, 3, 16, 16), (1, 3, 0, 16), (1, 2, 16, 16)):
        y = torch.zeros(shape, dtype=torch.float32, device="cuda:0")
        with pytest.raises(L.IDQError) as e:
            ctx.solve(y, tau=0.17, conv_prec="bf16")
        assert e.value.code == L.IDQ_E_INVAL, shape
        with pytest.raises(L.IDQError):
            ctx.grad_reg(y, conv_prec="f32")
    with pytest.raises(L.IDQError) as e:
        ctx.profile(True, every=0)
    assert e.value.code == L.IDQ_E_INVAL


def test_profile_sampling_times_one_launch_in_every():
    """Sampling every 5th launch of a class: 12 passes of each 64->64 class
    give launches 1, 6 and 11 timed, with their pixels counted."""
    layers = net_layers("rgb64", 0)
    taps, y = _deblur_batch(2, 40, 56)
    ctx = _ctx(layers, "blur", taps)
    yb = to_gpu(y, torch.float32)
    ctx.profile(True, classes=["conv64_bf16", "conv64_f32"], every=5)
    for _ in range(2):
        ctx.grad_reg(yb, conv_prec="bf16")
        ctx.grad_reg(yb, conv_prec="f32")
    prof = ctx.profile_read()
    ctx.profile(False)
    for cls in ("conv64_bf16", "conv64_f32"):
        assert prof[cls][1] == 3, (cls, prof[cls])
        assert prof[cls][2] == 3 * 2 * 40 * 56
    assert prof["conv_other"][1] == 0
