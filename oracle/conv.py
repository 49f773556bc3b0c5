"""3x3 convolution layers of the regularizer network N_theta, float64.

The network's layers are zero-padded "same" 3x3 cross-correlations with bias
(the convention of common deep-learning libraries). The paper's networks use
SoftPlus activations for RGB problems (Sec. 3.3; App. C), which is what these
functions provide.

Array layout: (n, c, h, w) float64; weights (c_out, c_in, 3, 3); bias (c_out,).
Pins: the adjoint identity <conv(x), d> = <x, conv_adjoint(d)>, agreement of
``conv3x3`` with torch.nn.functional.conv2d on CPU, and central differences of
the weight gradient (tests/test_oracle_conv.py).
"""
import numpy as np

TAPS = [(dy, dx) for dy in range(3) for dx in range(3)]


def conv3x3(x, W, b=None):
    """out[n,o,i,j] = b[o] + sum_{c,dy,dx} W[o,c,dy,dx] * x[n,c,i+dy-1,j+dx-1],
    with x taken as zero outside the image."""
    n, ci, h, w = x.shape
    co = W.shape[0]
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((n, co, h * w))
    for dy, dx in TAPS:
        shifted = xp[:, :, dy:dy + h, dx:dx + w].reshape(n, ci, h * w)
        out += np.matmul(np.ascontiguousarray(W[:, :, dy, dx]), shifted)
    out = out.reshape(n, co, h, w)
    if b is not None:
        out += b[None, :, None, None]
    return out


def conv3x3_adjoint(d, W):
    """Adjoint of the linear part of :func:`conv3x3` (the transposed conv):
    out[n,c,p,q] = sum_{o,dy,dx} W[o,c,dy,dx] * d[n,o,p-dy+1,q-dx+1].
    Implemented as the literal scatter of each tap's contribution."""
    n, co, h, w = d.shape
    ci = W.shape[1]
    outp = np.zeros((n, ci, h + 2, w + 2))
    dm = d.reshape(n, co, h * w)
    for dy, dx in TAPS:
        contrib = np.matmul(np.ascontiguousarray(W[:, :, dy, dx].T), dm).reshape(n, ci, h, w)
        outp[:, :, dy:dy + h, dx:dx + w] += contrib
    return outp[:, :, 1:h + 1, 1:w + 1]


def conv3x3_wgrad(g, x):
    """Gradient of sum(g * conv3x3(x, W)) w.r.t. W and b:
    dW[o,c,dy,dx] = sum_{n,i,j} g[n,o,i,j] * x[n,c,i+dy-1,j+dx-1],
    db[o] = sum_{n,i,j} g[n,o,i,j]."""
    n, co, h, w = g.shape
    ci = x.shape[1]
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    gm = g.reshape(n, co, h * w)
    dW = np.zeros((co, ci, 3, 3))
    for dy, dx in TAPS:
        shifted = xp[:, :, dy:dy + h, dx:dx + w].reshape(n, ci, h * w)
        dW[:, :, dy, dx] = sum(gm[i] @ shifted[i].T for i in range(n))
    return dW, gm.sum(axis=(0, 2))


def softplus(t):
    """SoftPlus with beta = 1 and no linear threshold:
    log(1 + e^t) = max(t, 0) + log1p(e^{-|t|})."""
    return np.maximum(t, 0.0) + np.log1p(np.exp(-np.abs(t)))


def sigmoid(t):
    """Derivative of softplus, 1 / (1 + e^{-t}), evaluated without overflow."""
    e = np.exp(-np.abs(t))
    return np.where(t >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def activation(name):
    """(sigma, sigma', sigma'') for an activation name ('softplus'|'identity')."""
    if name == "softplus":
        return (softplus, sigmoid,
                lambda t: sigmoid(t) * (1.0 - sigmoid(t)))
    if name == "identity":
        return (lambda t: t, lambda t: np.ones_like(t),
                lambda t: np.zeros_like(t))
    raise ValueError(name)
