"""The allocation-free entry point idq_grad_data_noalloc against idq_grad_data.

Both run the same stencil kernels; the no-alloc one stages its intermediate
image in the library's fixed per-GPU scratch array.  Two calls in a row, the
second on a smaller input, must each equal the allocating call's result
exactly (same kernels, same operands, same order of operations).
"""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, to_gpu
from paper_2605_19705_amd import IDQ, _lib as L

pytestmark = pytest.mark.gpu

OPS = {
    "blur9": dict(op_kind="blur", taps=synth.gaussian_taps(9, 1.6)),
    "tanh7": dict(op_kind="tanh_blur", taps=synth.uniform_taps(7), gain=2.0),
    "asym5": dict(op_kind="blur", taps=np.arange(1.0, 26.0).reshape(5, 5) / 325.0),
    "identity": dict(op_kind="identity"),
}


def _pair(shape, dtype, seed):
    x = to_gpu(synth.random_field(seed, shape), dtype)
    y = to_gpu(synth.random_field(seed + 1, shape), dtype)
    return x, y


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("op", list(OPS))
def test_noalloc_equals_allocating_call_twice(op, dtype):
    print(f"noalloc: op={op} dtype={dtype}", flush=True)
    ctx = IDQ(None, **OPS[op], device=0)
    for shape, seed in (((8, 3, 256, 256), 11), ((2, 3, 37, 45), 12)):
        x, y = _pair(shape, dtype, seed)
        ref = ctx.grad_data(x, y)
        out = torch.full_like(x, float("nan"))
        ctx.grad_data_noalloc(x, y, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (op, shape)
    ctx.close()


def test_noalloc_rejects_inputs_beyond_the_scratch():
    ctx = IDQ(None, **OPS["blur9"], device=0)
    # 2 * 3 * 1024 * 1024 float64 values = 48 MiB > the 32 MiB scratch: the
    # size check on the host refuses before any kernel is launched
    shape = (2, 3, 1024, 1024)
    x = torch.zeros(shape, dtype=torch.float64, device=dev())
    out = torch.empty_like(x)
    code = L.lib().idq_grad_data_noalloc(ctx._h, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()),
                                         C.c_void_p(out.data_ptr()), *shape, L.IDQ_F64, None)
    assert code == L.IDQ_E_INVAL
    assert b"scratch" in L.lib().idq_last_error()
    # identity needs no scratch: any size is accepted
    ctx2 = IDQ(None, op_kind="identity", device=0)
    y = torch.ones_like(x)
    ctx2.grad_data_noalloc(x, y, out)
    torch.cuda.synchronize()
    assert torch.equal(out, -y)
    ctx.close()
    ctx2.close()
