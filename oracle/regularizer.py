"""The learned explicit regularizer g_theta(x) = 1/2 ||x - N_theta(x)||^2 of the
gradient-step denoiser D = Id - grad g (Sec. 2.2, eq. GS), float64.

N_theta is a plain stack of 3x3 conv layers (list of (W, b)) with an
activation after every layer but the last.  If the network's input channel
count is 1 and the image has c > 1 channels, N is applied to each channel as
a separate grey image (the per-channel reading used for the 3-channel
nonlinear workload).

Recurrences (a_0 = x, h_l = W_l * a_{l-1} + b_l, a_l = sigma(h_l), N = h_L,
r = x - N):
  gradient   delta_L = r, delta_{l-1} = sigma'(h_{l-1}) . W_l^T delta_l,
             grad g = r - W_1^T delta_1                     (grad of eq. GS)
  HVP along w (forward-over-reverse):
             a'_0 = w, h'_l = W_l * a'_{l-1}, a'_l = sigma'(h_l) h'_l,
             r' = w - h'_L, delta'_L = r',
             delta'_{l-1} = sigma''(h_{l-1}) h'_{l-1} . W_l^T delta_l
                          + sigma'(h_{l-1}) . W_l^T delta'_l,
             H_g w = r' - W_1^T delta'_1
  parameter gradients
             dg/dW_l = -(delta_l corr a_{l-1}),  dg/db_l = -sum delta_l
             d/dtheta <u, grad_x g> (the mixed derivative, by symmetry of
             second derivatives the directional derivative of dg/dtheta
             along u):  W_l: -(delta'_l corr a_{l-1} + delta_l corr a'_{l-1}),
                        b_l: -sum delta'_l   (tangents taken with w = u)
Pins: central differences of g, grad g and the mixed derivative, Hessian
symmetry, the linear-network special case (tests/test_oracle_regularizer.py).
"""
import numpy as np

from .conv import conv3x3, conv3x3_adjoint, conv3x3_wgrad, activation


class Net:
    """Conv net N_theta: ``layers`` = list of (W, b) float64, ``act`` name."""

    def __init__(self, layers, act="softplus"):
        self.layers = [(np.asarray(W, np.float64), np.asarray(b, np.float64))
                       for W, b in layers]
        self.act = act
        self.c_in = self.layers[0][0].shape[1]
        self.c_out = self.layers[-1][0].shape[0]
        if self.c_in != self.c_out:
            raise ValueError("N must map images to images")

    @property
    def n_layers(self):
        return len(self.layers)

    def pack(self):
        """Flat parameter vector [W_1, b_1, W_2, b_2, ...] (C order)."""
        return np.concatenate([np.concatenate([W.ravel(), b.ravel()])
                               for W, b in self.layers])

    def with_params(self, flat):
        out, o = [], 0
        for W, b in self.layers:
            nW, nb = W.size, b.size
            out.append((flat[o:o + nW].reshape(W.shape), flat[o + nW:o + nW + nb].copy()))
            o += nW + nb
        return Net(out, self.act)

    # -- per-channel view ----------------------------------------------------
    def _to_net(self, x):
        n, c, h, w = x.shape
        if c == self.c_in:
            return x
        if self.c_in == 1:
            return x.reshape(n * c, 1, h, w)
        raise ValueError(f"image has {c} channels, net expects {self.c_in}")

    @staticmethod
    def _from_net(t, shape):
        return t.reshape(shape)

    # -- forward ---------------------------------------------------------------
    def forward(self, x):
        """Returns (hs, as_) with hs[l] = h_{l+1}, as_[l] = a_l (a_0 = x)."""
        sig, _, _ = activation(self.act)
        a = x
        hs, as_ = [], [x]
        L = self.n_layers
        for l, (W, b) in enumerate(self.layers):
            h = conv3x3(a, W, b)
            hs.append(h)
            if l < L - 1:
                a = sig(h)
                as_.append(a)
        return hs, as_

    def N(self, x):
        shape = x.shape
        hs, _ = self.forward(self._to_net(x))
        return self._from_net(hs[-1], shape)

    def g(self, x):
        """Per-image g(x) = 1/2 ||x - N(x)||^2, shape (n,)."""
        r = x - self.N(x)
        return 0.5 * np.sum(r * r, axis=(1, 2, 3))

    def _backward(self, hs, r):
        """deltas[l] = delta_{l+1} (delta_L = r) for l = 0..L-1."""
        _, dsig, _ = activation(self.act)
        L = self.n_layers
        deltas = [None] * L
        deltas[L - 1] = r
        for l in range(L - 1, 0, -1):
            W = self.layers[l][0]
            deltas[l - 1] = dsig(hs[l - 1]) * conv3x3_adjoint(deltas[l], W)
        return deltas

    def grad(self, x):
        """grad g(x) = r - J_N(x)^T r with r = x - N(x)."""
        shape = x.shape
        xn = self._to_net(x)
        hs, _ = self.forward(xn)
        r = xn - hs[-1]
        deltas = self._backward(hs, r)
        jtr = conv3x3_adjoint(deltas[0], self.layers[0][0])
        return self._from_net(r - jtr, shape)

    def _tangents(self, xn, hs, w):
        """Forward tangents along w: (hdots, adots) with adots[0] = w."""
        _, dsig, _ = activation(self.act)
        L = self.n_layers
        ad = w
        hdots, adots = [], [w]
        for l, (W, _) in enumerate(self.layers):
            hd = conv3x3(ad, W, None)
            hdots.append(hd)
            if l < L - 1:
                ad = dsig(hs[l]) * hd
                adots.append(ad)
        return hdots, adots

    def _second(self, xn, w):
        """Everything the HVP and mixed derivative need at (xn, w)."""
        _, dsig, d2sig = activation(self.act)
        hs, as_ = self.forward(xn)
        r = xn - hs[-1]
        deltas = self._backward(hs, r)
        hdots, adots = self._tangents(xn, hs, w)
        rdot = w - hdots[-1]
        L = self.n_layers
        ddots = [None] * L
        ddots[L - 1] = rdot
        for l in range(L - 1, 0, -1):
            W = self.layers[l][0]
            ddots[l - 1] = (d2sig(hs[l - 1]) * hdots[l - 1] * conv3x3_adjoint(deltas[l], W)
                            + dsig(hs[l - 1]) * conv3x3_adjoint(ddots[l], W))
        return hs, as_, r, deltas, hdots, adots, rdot, ddots

    def hvp(self, x, w):
        """H_g(x) w, the Hessian of g applied to w."""
        shape = x.shape
        xn, wn = self._to_net(x), self._to_net(w)
        _, _, _, _, _, _, rdot, ddots = self._second(xn, wn)
        out = rdot - conv3x3_adjoint(ddots[0], self.layers[0][0])
        return self._from_net(out, shape)

    def param_grad(self, x):
        """d/dtheta of sum over the batch of g(x): list of (dW, db)."""
        xn = self._to_net(x)
        hs, as_ = self.forward(xn)
        r = xn - hs[-1]
        deltas = self._backward(hs, r)
        out = []
        for l in range(self.n_layers):
            dW, db = conv3x3_wgrad(deltas[l], as_[l])
            out.append((-dW, -db))
        return out

    def mixed_grad(self, x, u):
        """d/dtheta <u, grad_x g(x; theta)> summed over the batch: list of
        (dW, db), from the tangent recurrences with w = u."""
        xn, un = self._to_net(x), self._to_net(u)
        hs, as_, r, deltas, hdots, adots, rdot, ddots = self._second(xn, un)
        out = []
        for l in range(self.n_layers):
            dW1, db1 = conv3x3_wgrad(ddots[l], as_[l])
            dW2, _ = conv3x3_wgrad(deltas[l], adots[l])
            out.append((-(dW1 + dW2), -db1))
        return out


def pack_grads(grads):
    """Flatten a list of (dW, db) like :meth:`Net.pack`."""
    return np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in grads])
