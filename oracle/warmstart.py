"""Warm-start network x^0 = y + W_phi(y), float64 (not part of the paper: a
learned initial iterate for the fixed-point iteration, which Alg. 1 allows by
taking any x^0).

Architecture (2-level conv encoder-decoder, 3x3 zero-padded convs, SoftPlus):
    e1 = sp(conv(y; 3->32)),  e2 = sp(conv(e1; 32->32))            full res
    p  = avgpool2x2(e2)                                            half res
    e3..e6 = sp(conv(.; 32->64)), sp(conv(.; 64->64)) x 3           half res
    u  = nearest-upsample2x(e6)                                    full res
    c  = concat(u, e2)            (64 + 32 = 96 channels, u first)
    d1 = sp(conv(c; 96->32)), d2 = sp(conv(d1; 32->32)), o = conv(d2; 32->3)
    x0 = y + o
Image height and width must be even.  Loss: mean squared error over all
elements.  Optimiser: Adam with bias correction (beta1 0.9, beta2 0.999,
eps 1e-8), the PyTorch defaults the paper trains with (App. D.1.3).
Pins (tests/test_oracle_warmstart.py): central differences of the loss; the
Adam step by closed forms (first step, a constant gradient over many steps,
a gradient followed by a zero gradient).
"""
import numpy as np

from .conv import conv3x3, conv3x3_adjoint, conv3x3_wgrad, softplus, sigmoid


def avgpool2(x):
    n, c, h, w = x.shape
    return x.reshape(n, c, h // 2, 2, w // 2, 2).mean(axis=(3, 5))


def avgpool2_adjoint(g):
    return np.repeat(np.repeat(g, 2, axis=2), 2, axis=3) * 0.25


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def upsample2_adjoint(g):
    n, c, h, w = g.shape
    return g.reshape(n, c, h // 2, 2, w // 2, 2).sum(axis=(3, 5))


def forward(layers, y):
    """Returns (x0, cache). ``layers`` is a list of 9 (W, b) pairs."""
    hs = []

    def conv(a, l):
        h = conv3x3(a, *layers[l])
        hs.append(h)
        return h

    e1 = softplus(conv(y, 0))
    e2 = softplus(conv(e1, 1))
    p = avgpool2(e2)
    e3 = softplus(conv(p, 2))
    e4 = softplus(conv(e3, 3))
    e5 = softplus(conv(e4, 4))
    e6 = softplus(conv(e5, 5))
    u = upsample2(e6)
    c = np.concatenate([u, e2], axis=1)
    d1 = softplus(conv(c, 6))
    d2 = softplus(conv(d1, 7))
    o = conv(d2, 8)
    ins = [y, e1, p, e3, e4, e5, c, d1, d2]
    return y + o, dict(hs=hs, ins=ins)


def backward(layers, cache, gout):
    """Gradients of sum(gout * x0) w.r.t. every (W, b)."""
    hs, ins = cache["hs"], cache["ins"]
    grads = [None] * 9

    def back(l, g):
        grads[l] = conv3x3_wgrad(g, ins[l])
        return conv3x3_adjoint(g, layers[l][0])

    g = back(8, gout)                       # d2
    g = back(7, g * sigmoid(hs[7]))         # d1
    g = back(6, g * sigmoid(hs[6]))         # c
    gu, ge2 = g[:, :64], g[:, 64:]
    g = upsample2_adjoint(gu)               # e6
    g = back(5, g * sigmoid(hs[5]))         # e5
    g = back(4, g * sigmoid(hs[4]))         # e4
    g = back(3, g * sigmoid(hs[3]))         # e3
    g = back(2, g * sigmoid(hs[2]))         # p
    ge2 = ge2 + avgpool2_adjoint(g)
    g = back(1, ge2 * sigmoid(hs[1]))       # e1
    back(0, g * sigmoid(hs[0]))             # y (input gradient unused)
    return grads


def mse_loss_grad(layers, y, target):
    """(loss, grads) for loss = mean((x0 - target)^2)."""
    x0, cache = forward(layers, y)
    diff = x0 - target
    loss = float(np.mean(diff * diff))
    gout = 2.0 * diff / diff.size
    return loss, backward(layers, cache, gout)


class Adam:
    """Adam (Kingma & Ba) with bias correction on a flat float64 vector."""

    def __init__(self, n, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, p, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return p - self.lr * mhat / (np.sqrt(vhat) + self.eps)
