"""Train the learned warm start x0 = y + W_phi(y) on fixed points the solver
itself produces (deblurring problem: circular 9x9 Gaussian blur, sigma 1.6,
noise 0.01, 5-layer 64-channel SoftPlus regularizer with seed-0 He-normal
weights, lambda 1, beta 0.5).

    python -m paper_2605_19705_amd.train_warmstart --out stage1.npy
    python -m paper_2605_19705_amd.train_warmstart --out stage2.npy \
        --init stage1.npy --lr 1e-3 --lr-min 1e-5
    ...

(the packaged weights: 60-epoch stages, the first from the seeded
initialisation, each later one from the previous stage's result with peak
learning rates 3e-3, 1e-3, 5e-4, 3e-4, 2e-4, ..., decaying to 1/100)

Steps, all on the GPU through the library:
  1. ``--pairs`` synthetic 3 x size x size ground truths (generator id
     ``--cfg-id``, disjoint from the evaluation images), y = A x + 0.01 n;
  2. x* = float32 i-DEQ solve of each y to rel. residual ``--solve-tol``;
  3. Adam on the mean squared error between y + W_phi(y) and x*, bf16 convs
     with float32 master weights (idq_ws_train_step), cosine learning-rate
     decay, the last ``--val`` pairs held out.
Writes the trained parameters (float32, packed [W_1, b_1, ..., W_9, b_9]).
"""
import argparse
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_2605_19705_amd import IDQ, WarmStart  # noqa: E402

NOISE = 0.01


def log(msg):
    print(msg, flush=True)


def deblur_context(device=0):
    layers = synth.he_normal_net(synth.net_channels("rgb64"), 0)
    taps = synth.gaussian_taps(9, 1.6)
    return IDQ(layers, op_kind="blur", taps=taps, device=device)


def measurements(ctx, cfg_id, first, n, size, dev):
    xt, nz = synth.make_batch(cfg_id, n, 3, size, size, first=first)
    x = torch.from_numpy(xt).float().to(dev)
    y = ctx.apply_A(x) + NOISE * torch.from_numpy(nz).float().to(dev)
    return y.contiguous()


def solver_pairs(ctx, n_pairs, size, cfg_id, batch, tol, dev, max_iter=1000):
    """(y, x*) on the GPU, x* from float32 solves started at y.  Images whose
    solve does not reach ``tol`` within ``max_iter`` are dropped and replaced by
    further images of the generator."""
    ys = torch.empty((n_pairs, 3, size, size), dtype=torch.float32, device=dev)
    xs = torch.empty_like(ys)
    y0 = measurements(ctx, cfg_id, 0, min(batch, n_pairs), size, dev)
    v0 = torch.from_numpy(synth.random_field(12345, tuple(y0.shape))).float().to(dev)
    L = ctx.lipschitz(y0, y0, v0, lam=1.0, iters=30, conv_prec="f32")
    tau = 0.9 / L
    log(f"pairs: L = {L:.5f}, tau = {tau:.5f}")
    t0 = time.perf_counter()
    iters, have, first, dropped = [], 0, 0, 0
    while have < n_pairs:
        n = batch
        y = measurements(ctx, cfg_id, first, n, size, dev)
        first += n
        x, res = ctx.solve(y, beta=0.5, tau=tau, lam=1.0, tol=tol, max_iter=max_iter,
                           conv_prec="f32")
        ok = np.nonzero(res.status == 0)[0]
        dropped += n - ok.size
        ok = ok[:n_pairs - have]
        idx = torch.from_numpy(ok).to(dev)
        ys[have:have + ok.size] = y.index_select(0, idx)
        xs[have:have + ok.size] = x.index_select(0, idx)
        have += ok.size
        iters.extend(res.iters[ok].tolist())
        log(f"pairs: {have}/{n_pairs} solved ({dropped} dropped), mean iterations "
            f"{np.mean(iters):.1f}, {time.perf_counter() - t0:.1f} s")
    return ys, xs, tau


def mse(a, b):
    return float(torch.mean((a - b) ** 2))


def train(ws, ys, xs, n_val, epochs, batch, lr, lr_min, prec, seed):
    n_train = ys.shape[0] - n_val
    steps_per_epoch = n_train // batch
    total = steps_per_epoch * epochs
    gen = torch.Generator().manual_seed(seed)
    yv, xv = ys[n_train:], xs[n_train:]
    log(f"train: {n_train} pairs, {n_val} held out, batch {batch}, {epochs} epochs, "
        f"{total} steps; held-out MSE of x0 = y: {mse(yv, xv):.3e}")
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n_train, generator=gen).to(ys.device)
        losses = []
        for i in range(steps_per_epoch):
            idx = perm[i * batch:(i + 1) * batch]
            yb = ys.index_select(0, idx).contiguous()
            xb = xs.index_select(0, idx).contiguous()
            a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / max(total - 1, 1)))
            want = (i % 16) == 0
            l = ws.train_step(yb, xb, a, prec=prec, want_loss=want)
            if want:
                losses.append(l)
            step += 1
        val = 0.0
        for j in range(0, n_val, batch):
            yb = yv[j:j + batch].contiguous()
            val += mse(ws.forward(yb, prec=prec), xv[j:j + batch]) * yb.shape[0]
        val /= max(n_val, 1)
        log(f"train: epoch {ep + 1}/{epochs}, train MSE {np.mean(losses):.3e}, held-out MSE "
            f"{val:.3e}, {time.perf_counter() - t0:.1f} s")
    return val


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--pairs", type=int, default=4096)
    ap.add_argument("--val", type=int, default=256)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--cfg-id", type=int, default=21)
    ap.add_argument("--solve-batch", type=int, default=128)
    ap.add_argument("--solve-tol", type=float, default=1e-5)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lr-min", type=float, default=2e-5)
    ap.add_argument("--prec", default="bf16")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--init", default=None,
                    help="start from these parameters (.npy, packed like --out) instead of "
                         "the seeded initialisation")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    ctx = deblur_context()
    ys, xs, _ = solver_pairs(ctx, args.pairs, args.size, args.cfg_id, args.solve_batch,
                             args.solve_tol, dev)
    p0 = (np.load(args.init).astype(np.float64) if args.init
          else synth.warmstart_init(args.seed))
    ws = WarmStart(p0, device=0)
    train(ws, ys, xs, args.val, args.epochs, args.batch, args.lr, args.lr_min, args.prec,
          args.seed)
    p = ws.get_params().astype(np.float32)
    np.save(args.out, p)
    log(f"saved {p.size} parameters to {args.out}")


if __name__ == "__main__":
    main()
