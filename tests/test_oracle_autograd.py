"""Pin of oracle.regularizer against an independent implementation: the
gradient-step potential g(x) = 1/2 ||x - N(x)||^2 (eq. GS) written directly
with torch CPU float64 ops, differentiated by torch autograd.

The torch network below is built from the definition only: 3x3 zero-padded
convolutions with bias, SoftPlus (log(1 + e^t), written as logaddexp(t, 0))
after every layer except the last, N(x) the last layer's output.  Every
derivative the oracle computes by hand-written recurrences (grad g, the
Hessian-vector product, the parameter gradient and the mixed second
derivative d/dtheta <u, grad_x g>) is compared with autograd's.  A
misplaced activation (for example one after the last layer, applied
consistently in the oracle's forward pass and in its recurrences) changes
N(x) itself and fails here, which finite differences of the oracle against
itself cannot catch.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import synth
from oracle import regularizer as R


def torch_net(params, chans):
    """Unpack the flat [W_1, b_1, ...] vector into per-layer tensors (views)."""
    out, o = [], 0
    for cin, cout in zip(chans[:-1], chans[1:]):
        nW = cout * cin * 9
        W = params[o:o + nW].reshape(cout, cin, 3, 3)
        b = params[o + nW:o + nW + cout]
        out.append((W, b))
        o += nW + cout
    return out


def torch_N(x, layers):
    t = x
    for l, (W, b) in enumerate(layers):
        t = F.conv2d(t, W, b, padding=1)
        if l < len(layers) - 1:
            t = torch.logaddexp(t, torch.zeros_like(t))
    return t


def torch_g(x, layers):
    """Per-image g, shape (n,)."""
    r = x - torch_N(x, layers)
    return 0.5 * (r * r).sum(dim=(1, 2, 3))


CASES = [("gray16", (2, 1, 9, 8)), ("rgb64", (1, 3, 7, 6))]


@pytest.mark.parametrize("name,shape", CASES)
def test_oracle_net_matches_torch_autograd(name, shape, rng):
    chans = synth.net_channels(name)
    layers = synth.he_normal_net(chans, 5, bias_seed=11)
    net = R.Net(layers)
    flat = net.pack()
    x = rng.uniform(-0.5, 1.5, shape)
    u = rng.standard_normal(shape)

    p = torch.tensor(flat, dtype=torch.float64, requires_grad=True)
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    ut = torch.tensor(u, dtype=torch.float64)
    tl = torch_net(p, chans)

    # N(x) and g(x)
    Nt = torch_N(xt, tl)
    np.testing.assert_allclose(net.N(x), Nt.detach().numpy(), rtol=0, atol=1e-13)
    gt = torch_g(xt, tl)
    np.testing.assert_allclose(net.g(x), gt.detach().numpy(), rtol=1e-13)

    # grad_x g and dg/dtheta (summed over the batch) in one autograd call
    gx, gp = torch.autograd.grad(gt.sum(), (xt, p), create_graph=True)
    scale = float(gx.detach().abs().max())
    np.testing.assert_allclose(net.grad(x), gx.detach().numpy(), rtol=0, atol=1e-12 * scale)
    pg = R.pack_grads(net.param_grad(x))
    np.testing.assert_allclose(pg, gp.detach().numpy(), rtol=0,
                               atol=1e-12 * float(gp.detach().abs().max()))

    # H_g u and d/dtheta <u, grad_x g> from the second derivative of <u, grad_x g>
    inner = (gx * ut).sum()
    hx, hp = torch.autograd.grad(inner, (xt, p))
    np.testing.assert_allclose(net.hvp(x, u), hx.numpy(), rtol=0,
                               atol=1e-12 * float(hx.abs().max()))
    mg = R.pack_grads(net.mixed_grad(x, u))
    np.testing.assert_allclose(mg, hp.numpy(), rtol=0, atol=1e-12 * float(hp.abs().max()))


def test_per_channel_grey_net_matches_torch(rng):
    """The grey net on a 3-channel image is the grey net on each channel."""
    chans = synth.net_channels("gray16")
    layers = synth.he_normal_net(chans, 2, bias_seed=4)
    net = R.Net(layers)
    x = rng.uniform(0, 1, (2, 3, 6, 7))
    p = torch.tensor(net.pack(), dtype=torch.float64)
    xt = torch.tensor(x.reshape(6, 1, 6, 7), dtype=torch.float64, requires_grad=True)
    g = torch_g(xt, torch_net(p, chans)).sum()
    (gx,) = torch.autograd.grad(g, xt)
    np.testing.assert_allclose(net.grad(x), gx.numpy().reshape(x.shape), rtol=0, atol=1e-12)


def test_misplaced_activation_is_caught(rng):
    """An oracle variant with SoftPlus after the last layer too (consistent in
    its forward pass and recurrences) disagrees with the torch definition."""
    chans = synth.net_channels("gray16")
    layers = synth.he_normal_net(chans, 5, bias_seed=11)

    class AllAct(R.Net):
        def forward(self, x):
            from oracle.conv import conv3x3, softplus
            a, hs, as_ = x, [], [x]
            for W, b in self.layers:
                h = conv3x3(a, W, b)
                hs.append(softplus(h))
                a = softplus(h)
                as_.append(a)
            return hs, as_[:-1]

    bad = AllAct(layers)
    x = rng.uniform(0, 1, (1, 1, 6, 6))
    p = torch.tensor(bad.pack(), dtype=torch.float64)
    Nt = torch_N(torch.tensor(x), torch_net(p, chans)).numpy()
    assert np.max(np.abs(bad.N(x) - Nt)) > 1e-3
