"""Gradients of a loss through the i-DEQ fixed point (App. D.1), float64.

At a fixed point xbar = T(xbar, xbar; Theta) of T(x1, x2) = z - tau grad F(z),
z = x1 + beta (x1 - x2), the two state Jacobians are
    dT/dx1 = (1 + beta)(I - tau H),  dT/dx2 = -beta (I - tau H),
with H = grad^2 F(xbar) symmetric, so the combined matrix of App. D.1.2 is
    I - dT/dx1 - dT/dx2 = tau H,
independent of beta (the second-argument derivative does not vanish by
itself; only the sum matters).  With v = dl/dxbar the adjoint u solves
    u = (I - tau H) u + v       (a fixed point; u* = (tau H)^{-1} v),
and
    dl/dtheta  = (dT/dtheta)^T u = -tau lambda d/dtheta <u, grad_x g(xbar)>
    dl/dlambda = -tau <grad g(xbar), u>
while d/dtau and d/dalpha vanish at an exact fixed point.
JFB (App. D.1.1) is the zero-iteration adjoint u = v.

Pins: a dense Hessian solve on tiny images and central differences of the
loss through tightly re-solved fixed points (tests/test_oracle_backward.py).
"""
import math

import numpy as np

from .regularizer import pack_grads


def adjoint_iterate(problem, xbar, y, v, tau, max_iter=500, tol=1e-8, beta=0.0):
    """Fixed-point iteration for u = (I - tau H) u + v started at u = v.

    With ``beta`` > 0 the same inertial extrapolation as the forward pass is
    applied to this linear map.  Stops when ||u_{j+1} - u_j|| / ||u_j|| < tol
    (batch 2-norms).  Returns (u, iterations, last relative change).
    """
    u = v.copy()
    up = v.copy()
    rel = math.inf
    j = 0
    for j in range(1, max_iter + 1):
        w = u + beta * (u - up)
        un = w - tau * problem.hvp(xbar, y, w) + v
        rel = math.sqrt(float(np.sum((un - u) ** 2)) / max(float(np.sum(u * u)), 1e-300))
        up, u = u, un
        if rel < tol:
            break
    return u, j, rel


def theta_grad(problem, xbar, y, u, tau):
    """(dl/dtheta packed like Net.pack, dl/dlambda) for a given adjoint u."""
    net, lam = problem.net, problem.lam
    mixed = pack_grads(net.mixed_grad(xbar, u))
    dtheta = -tau * lam * mixed
    dlam = -tau * float(np.sum(net.grad(xbar) * u))
    return dtheta, dlam


def dense_hessian(problem, x, y):
    """Dense Hessian of F at a single image x (1, c, h, w) from d HVPs."""
    d = x.size
    H = np.zeros((d, d))
    e = np.zeros(d)
    for i in range(d):
        e[:] = 0.0
        e[i] = 1.0
        H[:, i] = problem.hvp(x, y, e.reshape(x.shape)).ravel()
    return H
