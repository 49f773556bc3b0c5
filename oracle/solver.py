"""The i-DEQ forward pass: the inertial fixed-point iteration of Alg. 1, float64.

Objective (eq. inv_prob): F(x) = f(x, y) + lambda g(x).
One step of the i-DEQ operator (eq. ideq = RED step after eq. Momentum):
    z^k     = x^k + beta (x^k - x^{k-1})            beta = 1 - alpha
    x^{k+1} = z^k - tau (grad f(z^k, y) + lambda grad g(z^k))
The ``grad_at='current'`` variant evaluates the gradient at x^k instead
(heavy-ball form x^{k+1} = x^k + beta (x^k - x^{k-1}) - tau grad F(x^k)).
The proximal variant i-DEQ-P (App. B, eq. red_prox, Alg. 2) replaces the
gradient step on f by its proximal step:
    x^{k+1} = prox_{tau f(., y)}(z^k - tau lambda grad g(z^k)).
Its restart, stopping rule and averaging are read as those of Alg. 1 (Alg. 2
writes the restart as x^{k-1} <- x^k only; with B = inf, as everywhere here,
the two forms coincide).

Readings of Alg. 1 taken here (each image of a batch is an independent run):
  * x^{-1} = x^0, so the first step has no inertia.
  * after each update k <- k + 1 and S <- S + ||x^{k} - x^{k-1}||^2; if
    k * S > B^2 (strict, eq. restart) the inertia restarts: x^{-1} = x^0 =
    current iterate, k <- 0, S <- 0, so the next step has zero momentum.
    B = inf switches restart off.
  * stopping rule (App. D.1.3): ||x^{k+1} - x^k|| / ||x^k|| < tol per image
    (2-norm over all of the image's c*h*w values, strict), checked after every
    update; a converged image is frozen and its last iterate returned.
    If ||x^k|| = 0 the ratio is taken as 0 when x did not move, +inf otherwise.
  * ``fixed_iters = K`` performs exactly K updates x^1..x^K (no tolerance).
  * optional averaging step (Alg. 1, with Remark 1 noting it may be omitted):
    K_0 = argmin over floor(K/2) < k < K-1 of ||x^{k+1} - x^k|| (smallest k
    on ties), output (K_0 + 1)^{-1} sum_{k=0}^{K_0} z^k; only with
    ``fixed_iters`` and without restarts.
  * a non-finite iterate stops that image with status NONFINITE.
Parity pins: exact two-root trajectories on separable quadratics, the
per-frequency closed form for g = 0 with a circular blur, the dense solve of
the linear-network special case, restart indices on a quadratic
(tests/test_oracle_solver.py).
"""
import math

import numpy as np

CONVERGED, MAXITER, FIXED, NONFINITE = 0, 1, 2, -4


class Problem:
    """F(x) = f(x, y) + lambda g(x) for an operator (oracle.operators) and a
    regularizer net (oracle.regularizer.Net, or None for g = 0)."""

    def __init__(self, op, net, lam):
        self.op, self.net, self.lam = op, net, float(lam)

    def grad(self, x, y):
        gf = self.op.grad_f(x, y)
        if self.net is None or self.lam == 0.0:
            return gf
        return gf + self.lam * self.net.grad(x)

    def hvp(self, x, y, w):
        """Hessian of F at x along w: grad^2 f w + lambda H_g w."""
        hf = self.op.hess_f(x, y, w)
        if self.net is None or self.lam == 0.0:
            return hf
        return hf + self.lam * self.net.hvp(x, w)

    def value(self, x, y):
        v = self.op.f(x, y)
        if self.net is not None and self.lam != 0.0:
            v = v + self.lam * self.net.g(x)
        return v


def _sq(a):
    return np.sum(a * a, axis=tuple(range(1, a.ndim)))


def inertial_iterate(x0, grad_fn, beta, tau, tol=1e-4, max_iter=1000,
                     fixed_iters=None, restart_B=math.inf, grad_at="extrapolated",
                     averaging=False, record=False, prox_fn=None):
    """Alg. 1's forward loop for a batch of independent images.

    grad_fn(p, idx) returns grad F at points p for the images ``idx`` of the
    batch.  With ``prox_fn`` (Alg. 2) grad_fn returns lambda grad g only and
    the update is x^{k+1} = prox_fn(z - tau grad_fn(z, idx), idx).  Returns (x_out, info) where info holds per-image arrays
    ``iters``, ``rel`` (last relative residual), ``restarts``, ``status`` and,
    if ``record``, ``rels`` (list per image) and ``restart_at`` (global
    iteration counts after which a restart fired).
    """
    x0 = np.asarray(x0, dtype=np.float64)
    n = x0.shape[0]
    x = x0.copy()
    xprev = x0.copy()
    kr = np.zeros(n, dtype=np.int64)          # iterations since the last restart
    S = np.zeros(n)                           # restart accumulator
    it = np.zeros(n, dtype=np.int64)
    rel = np.full(n, np.inf)
    restarts = np.zeros(n, dtype=np.int64)
    status = np.full(n, MAXITER, dtype=np.int64)
    active = np.ones(n, dtype=bool)
    rels = [[] for _ in range(n)]
    restart_at = [[] for _ in range(n)]
    if averaging:
        if fixed_iters is None or math.isfinite(restart_B):
            raise ValueError("averaging needs fixed_iters and no restart")
        K = int(fixed_iters)
        zsum = np.zeros_like(x)
        best = np.full(n, np.inf)
        xhat = x0.copy()
    limit = fixed_iters if fixed_iters is not None else max_iter
    while active.any():
        idx = np.nonzero(active)[0]
        xa, xpa = x[idx], xprev[idx]
        z = xa + beta * (xa - xpa)
        p = z if grad_at == "extrapolated" else xa
        xn = z - tau * grad_fn(p, idx)
        if prox_fn is not None:
            xn = prox_fn(xn, idx)
        k_of = it[idx]                         # index k of this step (z^k -> x^{k+1})
        d2 = _sq(xn - xa)
        s0 = _sq(xa)
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.where(s0 > 0, np.sqrt(d2 / np.where(s0 > 0, s0, 1.0)),
                         np.where(d2 > 0, np.inf, 0.0))
        if averaging:
            zsum[idx] += z
            in_range = (k_of > K // 2) & (k_of < K - 1)
            better = in_range & (np.sqrt(d2) < best[idx])
            for j in np.nonzero(better)[0]:
                i = idx[j]
                best[i] = np.sqrt(d2[j])
                xhat[i] = zsum[i] / (k_of[j] + 1)
        xprev[idx], x[idx] = xa, xn
        it[idx] += 1
        kr[idx] += 1
        S[idx] += d2
        rel[idx] = r
        for j, i in enumerate(idx):
            if record:
                rels[i].append(float(r[j]))
            if not np.all(np.isfinite(xn[j])) or not np.isfinite(d2[j]):
                status[i] = NONFINITE
                active[i] = False
                continue
            if kr[i] * S[i] > restart_B ** 2:
                xprev[i] = x[i]
                kr[i] = 0
                S[i] = 0.0
                restarts[i] += 1
                if record:
                    restart_at[i].append(int(it[i]))
            if fixed_iters is not None:
                if it[i] >= fixed_iters:
                    status[i] = FIXED
                    active[i] = False
            elif r[j] < tol:
                status[i] = CONVERGED
                active[i] = False
            elif it[i] >= limit:
                status[i] = MAXITER
                active[i] = False
    out = xhat if averaging else x
    info = dict(iters=it, rel=rel, restarts=restarts, status=status)
    if record:
        info["rels"] = rels
        info["restart_at"] = restart_at
    return out, info


def ideq_solve(problem, y, x0, beta, tau, proximal=False, **kw):
    """i-DEQ forward pass on a batch: Alg. 1 with grad F = grad f + lambda grad g,
    or with ``proximal`` i-DEQ-P (Alg. 2): a gradient step on lambda g, then
    the proximal step of f."""
    y = np.asarray(y)
    if not np.iscomplexobj(y):
        y = y.astype(np.float64)
    if not proximal:
        def grad_fn(p, idx):
            return problem.grad(p, y[idx])

        return inertial_iterate(x0, grad_fn, beta, tau, **kw)
    if kw.get("grad_at", "extrapolated") != "extrapolated":
        raise ValueError("i-DEQ-P evaluates the gradient at z^k")

    def reg_fn(p, idx):
        if problem.net is None or problem.lam == 0.0:
            return np.zeros_like(p)
        return problem.lam * problem.net.grad(p)

    def prox_fn(v, idx):
        return problem.op.prox(v, y[idx], tau)

    return inertial_iterate(x0, reg_fn, beta, tau, prox_fn=prox_fn, **kw)


def power_iteration(problem, x, y, v0, iters=30):
    """Largest-magnitude eigenvalue of the batch Hessian of F at x.

    v <- v0 / ||v0||; repeat ``iters`` times: w = H v, L = <v, w>, v = w / ||w||.
    Returns the last Rayleigh quotient L (2-norms over the whole batch).
    The step size of the workloads is tau = 0.9 / L.
    """
    v = np.asarray(v0, dtype=np.float64)
    v = v / math.sqrt(float(np.sum(v * v)))
    L = 0.0
    for _ in range(iters):
        w = problem.hvp(x, y, v)
        L = float(np.sum(v * w))
        v = w / math.sqrt(float(np.sum(w * w)))
    return L
