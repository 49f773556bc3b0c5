"""The training loop of Alg. 1 (and Alg. 2 for i-DEQ-P), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One epoch of Alg. 1 over a dataset of pairs (y_i, x*_i), i < N:
  * gradient accumulator <- 0;
  * for every pair: the forward pass runs K updates of the i-DEQ iteration
    from x^0 (no tolerance; restart with threshold B; optionally the
    averaging step, whose output x_hat is the fixed-point estimate), then the
    gradient of the loss at x_hat is added to the accumulator;
  * one Adam step on Theta with the accumulated gradient.
Readings taken here:
  * the loss of an epoch is L = (1 / N) sum_i mean_pixels (x_hat_i - x*_i)^2,
    so dL/dx_hat_i = 2 (x_hat_i - x*_i) / (N d) with d = c h w;
  * JFB (App. D.1.1) takes the adjoint u = dL/dx_hat; the implicit mode solves
    u = (I - tau H_F(x_hat)) u + v by fixed-point iteration (oracle.backward);
    for i-DEQ-P the map is x -> P(z - tau lambda grad g(z)) with the linear
    part J_P = (I + tau A^T A)^{-1} of the proximal step, so JFB takes
    u = J_P v and the implicit adjoint solves u = (I - tau lambda H_g) J_P u + v
    and uses J_P u;
  * Theta = {theta, lambda} are trained; the derivatives with respect to tau
    and alpha vanish at an exact fixed point (App. D.1.2), so tau and beta stay
    at their initial values (the remark's bookkeeping);
  * Adam is oracle.warmstart.Adam (bias-corrected, float64), one instance for
    theta and one for lambda, with their own learning rates.
Pins: tests/test_oracle_training.py (the accumulated JFB gradient against the
closed form on a linear network; the implicit lambda-gradient against central
differences of the loss through dense fixed-point solves; the Adam step).
"""
import numpy as np

from . import backward as B
from . import solver as S
from .regularizer import pack_grads
from .warmstart import Adam


def prox_linear(op, v, tau):
    """J_P v = (I + tau A^T A)^{-1} v, the Jacobian of the proximal step."""
    return op.prox(v, np.zeros_like(op.A(v)), tau)


class Trainer:
    """Theta = (theta, lambda) with Adam states; ``net`` gives the layer shapes."""

    def __init__(self, net, op, lam, tau, beta, K, mode="jfb", lr_theta=1e-3, lr_lambda=1e-3,
                 learn_lambda=True, averaging=False, restart_B=np.inf, proximal=False,
                 adjoint_iters=500, adjoint_tol=1e-10):
        self.net, self.op = net, op
        self.theta = net.pack().copy()
        self.lam = float(lam)
        self.tau, self.beta, self.K = float(tau), float(beta), int(K)
        self.mode, self.learn_lambda = mode, learn_lambda
        self.averaging, self.restart_B, self.proximal = averaging, restart_B, proximal
        self.adjoint_iters, self.adjoint_tol = adjoint_iters, adjoint_tol
        self.opt_theta = Adam(self.theta.size, lr_theta)
        self.opt_lam = Adam(1, lr_lambda)

    def problem(self):
        return S.Problem(self.op, self.net.with_params(self.theta), self.lam)

    def forward(self, y, x0):
        P = self.problem()
        x, _ = S.ideq_solve(P, y, x0, self.beta, self.tau, proximal=self.proximal,
                            fixed_iters=self.K, restart_B=self.restart_B,
                            averaging=self.averaging)
        return x

    def gradient(self, xhat, y, v):
        """(dL/dtheta, dL/dlambda) at x_hat for dL/dx_hat = v."""
        P = self.problem()
        tau = self.tau
        if not self.proximal:
            if self.mode == "jfb":
                u = v
            else:
                u, _, _ = B.adjoint_iterate(P, xhat, y, v, tau, max_iter=self.adjoint_iters,
                                            tol=self.adjoint_tol)
            return B.theta_grad(P, xhat, y, u, tau)
        if self.mode == "jfb":
            w = prox_linear(self.op, v, tau)
        else:
            u = v.copy()
            for _ in range(self.adjoint_iters):
                w = prox_linear(self.op, u, tau)
                un = w - tau * self.lam * P.net.hvp(xhat, w) + v
                done = np.sqrt(np.sum((un - u) ** 2)) < self.adjoint_tol * np.sqrt(np.sum(u * u))
                u = un
                if done:
                    break
            w = prox_linear(self.op, u, tau)
        net = P.net
        dtheta = -tau * self.lam * pack_grads(net.mixed_grad(xhat, w))
        dlam = -tau * float(np.sum(net.grad(xhat) * w))
        return dtheta, dlam

    def epoch(self, Y, Xs, X0=None, batch=None):
        """One epoch of Alg. 1 over the N pairs (Y[i], Xs[i]); returns the loss
        (before the Adam step) and the accumulated (dtheta, dlambda)."""
        N = Y.shape[0]
        d = int(np.prod(Xs.shape[1:]))
        if X0 is None:      # from y; MRI data live in k-space: the zero-filled A^T y
            X0 = self.op.vjp(None, Y) if self.op.kind == "mri" else Y
        batch = N if batch is None else batch
        gth = np.zeros_like(self.theta)
        glam = 0.0
        loss = 0.0
        for s in range(0, N, batch):
            sl = slice(s, min(N, s + batch))
            xhat = self.forward(Y[sl], X0[sl])
            diff = xhat - Xs[sl]
            loss += float(np.sum(diff * diff)) / (N * d)
            v = 2.0 * diff / (N * d)
            dt, dl = self.gradient(xhat, Y[sl], v)
            gth += dt
            glam += dl
        self.theta = self.opt_theta.step(self.theta, gth)
        if self.learn_lambda:
            self.lam = float(self.opt_lam.step(np.array([self.lam]), np.array([glam]))[0])
        return loss, gth, glam
