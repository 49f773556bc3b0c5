"""GPU parity of the pixelwise and Fourier forward models against the oracle:
inpainting (App. D.3.2), Rician denoising (App. D.3.3) and real-valued MRI
(App. D.3.1): A, J_A^T, grad f, the Hessian of f, and the proximal step of f
(App. B, eq. red_prox) including the circular blur's; plus the inputs each
call refuses.

Tolerances: float64 1e-10 max-abs on values of order one (relative to the
largest magnitude where the values are large, as for the Rician gradient with
1 / sigma^2 = 400); float32 1e-4 on the same scale.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import to_gpu, to_np
from oracle import operators as O
from paper_2605_19705_amd import IDQ, _lib as L

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32}
TOL = {"f64": 1e-10, "f32": 1e-4}


def cdt(dt):
    return torch.complex128 if dt == torch.float64 else torch.complex64


def max_rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def make(kind, h, w, seed=3):
    if kind == "inpaint":
        m = synth.pixel_mask(seed, h, w, 0.5)
        return O.Operator("inpaint", mask=m), dict(op_kind="inpaint", mask=m)
    if kind == "mri":
        m = synth.cartesian_mask(seed, h, w, accel=4)
        return O.Operator("mri", mask=m), dict(op_kind="mri", mask=m)
    if kind == "mri_random":
        m = (np.random.default_rng(seed).random((h, w)) < 0.4).astype(float)
        return O.Operator("mri", mask=m), dict(op_kind="mri", mask=m)
    if kind == "rician":
        s = 25.5 / 255.0
        return O.Operator("rician", sigma=s), dict(op_kind="rician", sigma=s)
    if kind == "blur":
        k = np.random.default_rng(seed).uniform(0, 1, (5, 3))
        k /= k.sum()
        return O.Operator("blur", k), dict(op_kind="blur", taps=k)
    raise ValueError(kind)


def data(op, shape, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.2, 1.1, shape)
    if op.kind == "rician":
        y = np.abs(rng.uniform(0.0, 1.2, shape))
    else:
        y = op.A(rng.uniform(0, 1, shape))
        if np.iscomplexobj(y):
            y = y + 0.05 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
        else:
            y = y + 0.05 * rng.standard_normal(shape)
    v = rng.standard_normal(shape)
    return x, y, v


def gpu(a, dt):
    if np.iscomplexobj(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=cdt(dt))
    return to_gpu(a, dt)


SHAPES = [(2, 3, 16, 32), (1, 1, 64, 8), (3, 2, 4, 4)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["inpaint", "mri", "mri_random", "rician"])
def test_data_term_parity(kind, shape, prec):
    print(f"operators: {kind} {shape} {prec}", flush=True)
    dt = DT[prec]
    op, kw = make(kind, *shape[-2:])
    x, y, v = data(op, shape, 11)
    ctx = IDQ(None, **kw, device=0)
    xg, yg, vg = gpu(x, dt), gpu(y, dt), gpu(v, dt)
    tol = TOL[prec]
    assert max_rel(to_np(ctx.grad_data(xg, yg)), op.grad_f(x, y)) < tol
    assert max_rel(to_np(ctx.hvp(xg, vg, y=yg, lam=0.0, which="obj")),
                   op.hess_f(x, y, v)) < tol
    if kind != "rician":
        Ax = ctx.apply_A(xg)
        want = op.A(x)
        got = Ax.cpu().numpy().astype(np.complex128) if np.iscomplexobj(want) else to_np(Ax)
        assert max_rel(got, want) < tol
        assert max_rel(to_np(ctx.apply_AT(yg)), op.vjp(None, y)) < tol
        for tau in (0.3, 2.5):
            assert max_rel(to_np(ctx.prox_data(vg, yg, tau)), op.prox(v, y, tau)) < tol
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_blur_prox_parity(prec):
    dt = DT[prec]
    for shape in [(2, 3, 32, 16), (1, 1, 256, 256), (1, 2, 8, 4)]:
        op, kw = make("blur", *shape[-2:])
        x, y, v = data(op, shape, 5)
        ctx = IDQ(None, **kw, device=0)
        for tau in (0.2, 3.0):
            got = to_np(ctx.prox_data(gpu(v, dt), gpu(y, dt), tau))
            assert max_rel(got, op.prox(v, y, tau)) < TOL[prec], (shape, tau)
        ctx.close()


def test_rician_gradient_over_the_whole_argument_range():
    """t = x y / s^2 from 0 to ~1e4 crosses the series / expansion switch."""
    s = 0.05
    ctx = IDQ(None, op_kind="rician", sigma=s, device=0)
    op = O.Operator("rician", sigma=s)
    t = np.concatenate([[0.0, 1e-6, 0.5], np.linspace(1, 60, 1181), np.geomspace(60, 1e4, 200)])
    x = np.full(t.size, 0.9)
    y = t * s * s / 0.9
    shape = (1, 1, 1, t.size)
    for prec, tol in (("f64", 1e-13), ("f32", 2e-6)):
        dt = DT[prec]
        got = to_np(ctx.grad_data(to_gpu(x.reshape(shape), dt), to_gpu(y.reshape(shape), dt)))
        want = op.grad_f(x.reshape(shape), y.reshape(shape))
        # gradient values are differences of terms of size x / s^2 = 360 and y / s^2
        scale = np.maximum(0.9, y.reshape(shape)) / s ** 2
        assert float(np.max(np.abs(got - want) / scale)) < tol, prec
    ctx.close()


def test_operator_refusals():
    m = synth.pixel_mask(1, 8, 8)
    ctx = IDQ(None, op_kind="inpaint", mask=m, device=0)
    x = torch.zeros((1, 1, 8, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(L.IDQError) as e:            # mask size differs from the image's
        ctx.grad_data(x, x)
    assert e.value.code == L.IDQ_E_INVAL
    ctx.close()
    mm = synth.cartesian_mask(1, 12, 8, accel=4)
    with pytest.raises(L.IDQError) as e:            # 12 is not a power of two
        IDQ(None, op_kind="mri", mask=mm, device=0)
    assert e.value.code == L.IDQ_E_UNSUPPORTED
    with pytest.raises(L.IDQError) as e:            # masks hold 0 or 1
        IDQ(None, op_kind="inpaint", mask=0.5 * m, device=0)
    assert e.value.code == L.IDQ_E_INVAL
    ctx = IDQ(None, op_kind="mri", mask=synth.cartesian_mask(1, 8, 8, accel=4), device=0)
    x = torch.zeros((1, 1, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):                 # MRI data are complex
        ctx.grad_data(x, x)
    ctx.close()
    ctx = IDQ(None, op_kind="rician", sigma=0.1, device=0)
    x = torch.zeros((1, 1, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(L.IDQError) as e:            # no closed-form prox
        ctx.prox_data(x, x, 0.5)
    assert e.value.code == L.IDQ_E_UNSUPPORTED
    ctx.close()
    with pytest.raises(L.IDQError):
        IDQ(None, op_kind="rician", sigma=0.0, device=0)
