#!/usr/bin/env python
"""Throughput of the i-DEQ forward pass on one MI355X.

Workload (deblurring): a batch of 8 synthetic 3x256x256 images, circular 9x9
Gaussian blur (sigma 1.6) plus noise of std 0.01, regularizer
g(x) = 1/2 ||x - N(x)||^2 with N a 5-layer 3->64->64->64->64->3 SoftPlus conv
net (He-normal, seed 0), lambda 1, beta 0.5, tau = 0.9 / L with L from 30
power iterations at the measurements (computed once, outside the timed region).
One step = one i-DEQ solve of the whole batch until every image reaches
||x^{k+1} - x^k|| / ||x^k|| < 1e-4.

Two arms are timed:
  headline  bf16 matrix-core convs (fp32 accumulate) until rel < 2e-3 or
            stagnation, then split-bf16 convs (each float operand as bf16
            hi + lo, three products) to rel < 1e-4, then fp32 convs until an
            fp32 update has rel < 1e-4 (--refine f32 skips the split phase);
            started from the learned warm start when its weights are
            available (else from y),
  fp32      fp32 matrix-core convs from x0 = y ("FP32 plain").
Inside the timed region one launch in five of each 64->64 conv class carries
HIP events (its device time feeds the roofline figures).  After it: one solve
with every kernel class timed, the tanh-blur workload (16x3x128x128, fp32), the
4x3x512x512 batch from y, zero and the warm start, the i-DEQ-P inpainting,
Rician and i-DEQ-P MRI workloads (8 images of 256x256), training epochs of
Alg. 1, and the float64 oracle on the host.  Prints one JSON line (value =
headline images/s).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PROF_CLASSES = ["conv64_bf16", "conv64_f32", "conv_other", "stencil", "update", "warmstart",
                "conv64_bf16x3"]
METRIC = "restored 256^2 images/s at rel. residual 1e-4: BF16+warm-start vs FP32 plain"
BF16_PEAK = 2.5e15     # MI355X dense bf16 matrix-core peak, FLOP/s
F32_PEAK = 157.3e12    # MI355X dense fp32 matrix-core peak, FLOP/s
FLOP_PER_PX_64 = 2 * 9 * 64 * 64   # one 64->64 3x3 conv pass
# HBM bytes per output pixel of the 64->64 conv kernels in this solve, from
# the FETCH_SIZE / WRITE_SIZE counter runs summarised in profiles/ (FETCH x 2.0,
# WRITE x 1.0, the factors a 256 MiB device copy gives; bytes of the solve's
# launches over the pixels they computed).  `traffic` is this figure times the
# pixels per timed launch.  A figure is valid only while the kernel's device
# code is the one measured (sha256 of its sources), else it is reported as null.
TRAFFIC = {
    "conv64_bf16": {"bytes_per_px": 336.69,
                    "sha256": "2f12adc0dacffb85e211299a47045de1c257af3ce9f5872c4043d5a2e57ea122",
                    "sources": ("paper_2605_19705_amd/csrc/k_conv_mfma.h",
                                "paper_2605_19705_amd/csrc/k_conv_split64.h",
                                "paper_2605_19705_amd/csrc/k_conv_mfma_bf16.hip")},
    "conv64_bf16x3": {"bytes_per_px": 673.39,
                      "sha256": "093520476a45508be24cc7f27c22a9afca5b4ed3e8b8c36f741d801a64289580",
                      "sources": ("paper_2605_19705_amd/csrc/k_conv_mfma.h",
                                  "paper_2605_19705_amd/csrc/k_conv_split64.h",
                                  "paper_2605_19705_amd/csrc/k_conv_mfma_split.hip")},
}


def sources_sha256(sources):
    import hashlib
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_problem(torch, n=8, h=256, w=256):
    import synth
    from paper_2605_19705_amd import IDQ
    layers = synth.he_normal_net(synth.net_channels("rgb64"), 0)
    taps = synth.gaussian_taps(9, 1.6)
    ctx = IDQ(layers, op_kind="blur", taps=taps, device=0)
    xt, nz = synth.make_batch(2, n, 3, h, w)
    dev = torch.device("cuda:0")
    xt_g = torch.from_numpy(xt).float().to(dev)
    nz_g = torch.from_numpy(nz).float().to(dev)
    y = ctx.apply_A(xt_g) + 0.01 * nz_g
    return ctx, y.contiguous(), layers, taps, xt, nz


def time_arm(torch, ctx, y, K, W, profile=None, every=1, check=True, **kw):
    """W warm-up solves, then K timed solves; ``profile``: names of the kernel
    classes whose launches are timed by HIP events inside the timed region, one
    launch in ``every`` of each class."""
    for _ in range(W):
        ctx.solve(y, **kw)
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True, classes=profile, every=every)
    times, iters, low, mid, status = [], [], [], [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(K):
        t0 = time.perf_counter()
        x, res = ctx.solve(y, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        iters.append(res.iters.tolist())
        low.append(res.iters_low.tolist())
        mid.append(res.iters_mid.tolist())
        status.append(res.status.tolist())
        assert not check or (res.status == 0).all(), f"solve did not converge: {res.status}"
    total = time.perf_counter() - t_all
    prof = ctx.profile_read() if profile else None
    if profile:
        ctx.profile(False)
    return dict(total_s=total, step_s=times, iters=iters, iters_low=low, iters_mid=mid, prof=prof,
                x=x, status=status)


def also_measured(torch, poll, ws, head_ctx=None, head_y=None, head_tau=None):
    """The other workloads the headline's measurement plan names, timed briefly
    (1 warm-up + 2 timed solves each): the tanh-blur problem in fp32 and the
    4 x 3 x 512 x 512 deblurring batch from y, zero and the warm start; and the
    cost of one iteration of the headline batch in each arithmetic (10 fixed
    iterations, every image active, the bf16 run held in its phase)."""
    import synth
    from paper_2605_19705_amd import IDQ
    dev = torch.device("cuda:0")
    out = {}

    def batch(ctx, cfg_id, n, h, w):
        xt, nz = synth.make_batch(cfg_id, n, 3, h, w)
        y = ctx.apply_A(torch.from_numpy(xt).float().to(dev)) + \
            0.01 * torch.from_numpy(nz).float().to(dev)
        y = y.contiguous()
        v0 = torch.from_numpy(synth.random_field(12345, tuple(y.shape))).float().to(dev)
        return y, 0.9 / ctx.lipschitz(y, y, v0, lam=1.0, iters=30, conv_prec="f32")

    def summary(r, n):
        return {"images_per_s": n * len(r["step_s"]) / r["total_s"],
                "ms_per_solve": 1e3 * r["total_s"] / len(r["step_s"]),
                "iters_per_image": r["iters"][-1], "status": r["status"][-1]}

    log("bench: denoising 1x1x32x32, float64, 100 fixed updates")
    ctx1 = IDQ(synth.he_normal_net(synth.net_channels("gray16"), 0), op_kind="identity",
               device=0)
    xt1, nz1 = synth.make_batch(1, 1, 1, 32, 32)
    y1 = torch.from_numpy(xt1 + 25.0 / 255.0 * nz1).to(dev)
    v01 = torch.from_numpy(synth.random_field(12345, tuple(y1.shape))).to(dev)
    tau1 = 0.9 / ctx1.lipschitz(y1, y1, v01, lam=1.0, iters=30, conv_prec="f64")
    r = time_arm(torch, ctx1, y1, 5, 2, check=False, conv_prec="f64", beta=0.5, tau=tau1,
                 lam=1.0, fixed_iters=100, poll_every=100)
    out["denoise_1x1x32_f64_100_updates"] = dict(
        ms_per_solve=1e3 * r["total_s"] / len(r["step_s"]),
        us_per_update=1e4 * r["total_s"] / len(r["step_s"]),
        workload="A = identity, noise 25/255, 1->16->16->1 softplus net, float64, 100 updates "
                 "(launch-bound: 9 kernels per update on a 32x32 image)")
    del ctx1

    log("bench: tanh-blur workload (16x3x128x128, fp32)")
    ctx3 = IDQ(synth.he_normal_net(synth.net_channels("gray16"), 0), op_kind="tanh_blur",
               taps=synth.uniform_taps(7), device=0)
    y3, tau3 = batch(ctx3, 3, 16, 128, 128)
    r = time_arm(torch, ctx3, y3, 2, 1, check=False, conv_prec="f32", beta=0.5, tau=tau3,
                 lam=1.0, tol=1e-4, max_iter=2000, poll_every=poll)
    out["tanh_blur_16x3x128_fp32"] = dict(
        summary(r, 16), workload="A(x) = tanh(2 k*x) / tanh 2, 7x7 uniform k, noise 0.01, "
                                 "1->16->16->1 softplus net per channel, fp32 convs")
    del ctx3, y3

    log("bench: 4x3x512x512 deblurring from y, zero and the warm start")
    ctx5 = IDQ(synth.he_normal_net(synth.net_channels("rgb64"), 0), op_kind="blur",
               taps=synth.gaussian_taps(9, 1.6), device=0)
    y5, tau5 = batch(ctx5, 5, 4, 512, 512)
    kw = dict(beta=0.5, tau=tau5, lam=1.0, tol=1e-4, max_iter=3000, poll_every=poll,
              conv_prec="bf16", refine_prec="bf16x3", switch_tol=2e-3, switch_patience=5)
    res5 = {}
    for init in ("y", "zero") + (("warmstart",) if ws is not None else ()):
        extra = dict(ws=ws, ws_prec="bf16") if init == "warmstart" else {}
        res5[init] = summary(time_arm(torch, ctx5, y5, 2, 1, check=False, init=init, **kw,
                                      **extra), 4)
    out["deblur_4x3x512_by_init"] = res5

    if head_ctx is not None:
        per_it = {}
        for prec, extra in (("bf16", dict(switch_tol=0.0, switch_patience=1 << 30)),
                            ("bf16x3", {}), ("f32", {})):
            r = time_arm(torch, head_ctx, head_y, 2, 1, check=False, conv_prec=prec,
                         beta=0.5, tau=head_tau, lam=1.0, fixed_iters=10, poll_every=poll,
                         **extra)
            per_it[prec] = 1e3 * r["total_s"] / len(r["step_s"]) / 10
        out["ms_per_iteration_8x3x256_by_arithmetic"] = per_it
    return out


# Algorithmic bytes per pixel (float32) of one data-term call of the workloads
# below: the MRI gradient F^H M_s F z - A^T y (forward rows: z in, complex out;
# columns: complex in and out; inverse rows: complex and A^T y in, real out),
# the MRI proximal step (the same with z, the regularizer gradient and A^T y
# read by the forward rows), the inpainting proximal step (z, the regularizer
# gradient and y in, the result out; the mask is shared by the 3 channels) and
# the Rician gradient (x and y in, the gradient out).
DATA_TERM_BYTES_PER_PX = {"mri_grad": 44.0, "mri_prox": 48.0, "inpaint_prox": 16.0 + 4.0 / 3,
                          "rician_grad": 12.0}


def paper_workloads(torch, poll):
    """The paper's other data terms on 8 synthetic 256^2 images, each solved to
    rel 1e-4 in float32 and bf16 -> split-bf16 -> float32 (1 warm-up and 2 timed
    solves per arm), with the data term's device time and bandwidth from one
    more solve with every kernel class timed; and one training epoch of Alg. 1
    (16 pairs of 3 x 128^2, K = 100, JFB and implicit)."""
    import numpy as np
    import synth
    from paper_2605_19705_amd import IDQ, Trainer
    dev = torch.device("cuda:0")
    out = {}

    def tau_for(ctx, x0, y, lam):
        v0 = torch.from_numpy(synth.random_field(12345, tuple(x0.shape))).float().to(dev)
        return 0.9 / ctx.lipschitz(x0, y, v0, lam=lam, iters=30, conv_prec="f32")

    def run(name, ctx, y, x0, lam, beta, proximal, term, px):
        tau = tau_for(ctx, x0, y, lam)
        res = {"tau": tau, "lambda": lam, "beta": beta}
        kw = dict(beta=beta, tau=tau, lam=lam, tol=1e-4, max_iter=3000, poll_every=poll,
                  proximal=proximal, x0=x0)
        for arm, extra in (("f32", dict(conv_prec="f32")),
                           ("bf16_split_f32", dict(conv_prec="bf16", refine_prec="bf16x3",
                                                   switch_tol=2e-3, switch_patience=5))):
            r = time_arm(torch, ctx, y, 2, 1, check=False, **kw, **extra)
            res[arm] = {"images_per_s": y.shape[0] * len(r["step_s"]) / r["total_s"],
                        "ms_per_solve": 1e3 * r["total_s"] / len(r["step_s"]),
                        "iters_per_image": r["iters"][-1], "status": r["status"][-1]}
        cb = class_breakdown(torch, ctx, y, conv_prec="f32", **kw)["stencil"]
        if cb["launches"]:
            t = cb["ms"] / cb["launches"]
            byt = DATA_TERM_BYTES_PER_PX[term] * px
            res["data_term"] = {"call": term, "calls_one_solve": cb["launches"],
                                "avg_us": 1e3 * t, "algorithmic_bytes": byt,
                                "achieved_GBps": byt / (t * 1e-3) / 1e9,
                                "frac_of_hbm": byt / (t * 1e-3) / 8e12}
        out[name] = res

    log("bench: i-DEQ-P inpainting (8x3x256x256, 50% pixels, noise 5/255)")
    n, h, w = 8, 256, 256
    xt, nz = synth.make_batch(31, n, 3, h, w)
    m = synth.pixel_mask(31, h, w, 0.5)
    ctx = IDQ(synth.he_normal_net(synth.net_channels("rgb64"), 0), op_kind="inpaint", mask=m,
              device=0)
    y = (ctx.apply_A(torch.from_numpy(xt).float().to(dev)) +
         5.0 / 255.0 * torch.from_numpy(nz).float().to(dev)).contiguous()
    run("inpaint_8x3x256_ideq_p", ctx, y, y, 0.83, 0.8, True, "inpaint_prox", n * 3 * h * w)
    del ctx, y

    log("bench: Rician denoising (8x3x256x256, sigma 25.5/255)")
    s = 25.5 / 255.0
    xt, nz = synth.make_batch(33, n, 3, h, w)
    ni = synth.random_field(330, xt.shape)
    yr = np.sqrt((xt + s * nz) ** 2 + (s * ni) ** 2)
    ctx = IDQ(synth.he_normal_net(synth.net_channels("rgb64"), 0), op_kind="rician", sigma=s,
              device=0)
    y = torch.from_numpy(yr).float().to(dev).contiguous()
    run("rician_8x3x256", ctx, y, y, 6.0, 0.8, False, "rician_grad", n * 3 * h * w)
    del ctx, y

    log("bench: i-DEQ-P MRI x8 (8x1x256x256 k-space, noise 1/255)")
    xt, nz = synth.make_batch(32, n, 1, h, w)
    mk = synth.cartesian_mask(32, h, w, accel=8)
    ctx = IDQ(synth.he_normal_net(synth.net_channels("gray16"), 0), op_kind="mri", mask=mk,
              device=0)
    ni = synth.random_field(320, xt.shape)
    yk = ctx.apply_A(torch.from_numpy(xt).float().to(dev))
    noise = torch.complex(torch.from_numpy(nz).float(), torch.from_numpy(ni).float()).to(dev)
    y = (yk + (1.0 / 255.0) * torch.from_numpy(mk).float().to(dev) * noise).contiguous()
    x0 = ctx.apply_AT(y)
    run("mri_8x1x256_ideq_p", ctx, y, x0, 0.65, 0.8, True, "mri_prox", n * h * w)
    del ctx, y, x0

    log("bench: training epochs of Alg. 1 (16x3x128x128 deblurring pairs, K = 100)")
    xt, nz = synth.make_batch(4, 16, 3, 128, 128)
    taps = synth.gaussian_taps(9, 1.6)
    ctx = IDQ(synth.he_normal_net(synth.net_channels("rgb64"), 0), op_kind="blur", taps=taps,
              device=0)
    Xs = torch.from_numpy(xt).float().to(dev)
    Y = (ctx.apply_A(Xs) + 0.01 * torch.from_numpy(nz).float().to(dev)).contiguous()
    tau = tau_for(ctx, Y, Y, 1.0)
    tr_out = {"pairs": 16, "K": 100, "tau": tau}
    for mode, adj in (("jfb", 0), ("implicit", 20)):
        tr = Trainer(ctx, 1.0)
        kw = dict(K=100, beta=0.5, tau=tau, mode=mode, lr_theta=1e-4, lr_lambda=1e-3,
                  adjoint_max_iter=adj, adjoint_tol=0.0)
        tr.epoch(Y, Xs, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = [tr.epoch(Y, Xs, **kw) for _ in range(2)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 2
        # conv flops of the epoch's forward solves alone (K updates x one
        # regularizer gradient per pair: forward and transposed passes of the
        # 3->64->64->64->64->3 net), a lower bound on the epoch's flops
        fl = 100 * 2 * (2 * 9 * 3 * 64 * 2 + 3 * FLOP_PER_PX_64) * 16 * 128 * 128
        tr_out[mode] = {"s_per_epoch": dt, "pairs_per_s": 16 / dt, "adjoint_iters": adj,
                        "loss": losses, "forward_conv_flops": fl,
                        "achieved_TFLOPs": fl / dt / 1e12,
                        "frac_of_fp32_matrix_peak": fl / dt / F32_PEAK}
        tr.close()
    out["training_epoch_16x3x128_f32"] = tr_out

    log("bench: warm-start training steps (16x3x128x128 pairs, bf16, Adam)")
    from paper_2605_19705_amd import WarmStart
    ws = WarmStart(synth.warmstart_init(0), device=0)
    yb, tb = Y[:16].contiguous(), Xs[:16].contiguous()
    ws.train_step(yb, tb, 1e-4, prec="bf16", want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        ws.train_step(yb, tb, 1e-4, prec="bf16", want_loss=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 10
    # flops of one step: the forward pass, the backward pass and the weight
    # gradient, each ~ the network's conv flops (full resolution: 3->32, 32->32,
    # 96->32, 32->32, 32->3; half resolution: 32->64 and 3 x 64->64)
    fwd_px = 2 * 9 * (3 * 32 + 32 * 32 + 96 * 32 + 32 * 32 + 32 * 3) + \
        2 * 9 * (32 * 64 + 3 * 64 * 64) // 4
    fl = 3 * fwd_px * 16 * 128 * 128
    out["warmstart_train_step_16x3x128_bf16"] = {"ms_per_step": 1e3 * dt, "pairs_per_s": 16 / dt,
                                                 "params": ws.num_params, "conv_flops": fl,
                                                 "achieved_TFLOPs": fl / dt / 1e12,
                                                 "frac_of_bf16_peak": fl / dt / BF16_PEAK}
    return out


def class_breakdown(torch, ctx, y, **kw):
    """Device time per kernel class of one more solve (outside the timed region:
    timing every class adds an event pair to each launch)."""
    ctx.profile(True)
    ctx.solve(y, **kw)
    torch.cuda.synchronize()
    p = ctx.profile_read()
    ctx.profile(False)
    return {k: {"ms": v[0], "launches": v[1]} for k, v in p.items()}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(iters_per_image, sample_iters=10, repeats=3):
    """The float64 oracle on the host, as it stands: one 256x256 image of the
    headline batch, `sample_iters` i-DEQ iterations timed `repeats` times; the
    median time per image-iteration, scaled by the GPU fp32 arm's mean iteration
    count to rel 1e-4, gives images per second (the 8 images of the batch are
    independent, so the batch takes 8 times as long).  ``cores`` is the BLAS
    thread count the oracle's matrix products ran on."""
    import numpy as np
    import synth
    from oracle import operators as O, regularizer as R, solver as S
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    layers = synth.he_normal_net(synth.net_channels("rgb64"), 0)
    op = O.Operator("blur", synth.gaussian_taps(9, 1.6))
    xt, nz = synth.make_batch(2, 1, 3, 256, 256)
    y = op.A(xt) + 0.01 * nz
    P = S.Problem(op, R.Net(layers), 1.0)
    runs = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        S.ideq_solve(P, y, y, 0.5, 0.15, fixed_iters=sample_iters)
        runs.append(time.perf_counter() - t0)
    t_iter = float(np.median(runs)) / sample_iters
    return {"value": 1.0 / (t_iter * iters_per_image), "unit": "images/s", "cores": int(cores),
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"image 0 of the 8-image batch, {sample_iters} float64 i-DEQ iterations, "
                      f"median of {repeats} runs ({t_iter:.3f} s per image-iteration), scaled by "
                      f"the fp32 arm's {iters_per_image:.1f} iterations per image"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the fp32-plain arm")
    ap.add_argument("--refine", default="bf16x3", choices=["f32", "bf16x3"],
                    help="bf16x3: a split-bf16 phase between the bf16 phase and the float32 "
                         "updates that end every solve; f32: straight to float32")
    ap.add_argument("--switch-tol", type=float, default=2e-3,
                    help="bf16 phase ends when rel < this ...")
    ap.add_argument("--patience", type=int, default=5,
                    help="... or after this many bf16 updates without a new best rel")
    ap.add_argument("--poll", type=int, default=3,
                    help="solver iterations enqueued between host polls of the phases")
    ap.add_argument("--profile-all", action="store_true",
                    help="time every kernel class inside the timed region (slower)")
    ap.add_argument("--sample-every", type=int, default=5,
                    help="time one launch in this many of each timed class inside the timed "
                         "region (each timed launch holds the queue for its event packets)")
    ap.add_argument("--no-also", action="store_true",
                    help="skip the tanh-blur and 512^2 warm-start measurements")
    ap.add_argument("--no-paper-workloads", action="store_true",
                    help="skip the inpainting, Rician, MRI and training measurements")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy a buffer of this many MiB device-to-device (a plain copy "
                         "kernel of known size, for scaling hardware byte counters)")
    ap.add_argument("--ws-weights", default=os.path.join(ROOT, "paper_2605_19705_amd", "weights",
                                                         "warmstart_deblur.npy"),
                    help="trained warm-start parameters (.npy, packed [W_1, b_1, ...])")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the per-image solves need no exchange, so more "
              "GPUs would run independent shares of the batch; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth

    if args.copy_probe > 0:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy probe of {nbytes} bytes done")
        del src, dst

    log("bench: building the deblurring problem (8x3x256x256)")
    ctx, y, layers, taps, xt, nz = make_problem(torch)
    v0 = torch.from_numpy(synth.random_field(12345, tuple(y.shape))).float().to(y.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = ctx.lipschitz(y, y, v0, lam=1.0, iters=30, conv_prec="f32")
    t_L = time.perf_counter() - t0
    tau = 0.9 / L
    log(f"bench: L = {L:.6f}, tau = {tau:.6f} ({t_L * 1e3:.1f} ms, outside the timed region)")

    common = dict(beta=0.5, tau=tau, lam=1.0, tol=1e-4, max_iter=2000, poll_every=args.poll)
    ws = None
    init = "y"
    if args.ws_weights and os.path.exists(args.ws_weights):
        from paper_2605_19705_amd import WarmStart
        ws = WarmStart(np.load(args.ws_weights).astype(np.float64), device=0)
        init = "warmstart"
    head_kw = dict(common, conv_prec="bf16", switch_tol=args.switch_tol,
                   switch_patience=args.patience, init=init, ws=ws,
                   ws_prec="bf16", refine_prec=args.refine)

    log(f"bench: headline arm (bf16 + fp32 refinement, init={init}), "
        f"{args.warmup} warmup + {args.steps} timed solves")
    head = time_arm(torch, ctx, y, args.steps, args.warmup,
                    profile=PROF_CLASSES if args.profile_all else ["conv64_bf16", "conv64_bf16x3"],
                    every=args.sample_every, **head_kw)
    n_img = y.shape[0]
    value = n_img * args.steps / head["total_s"]
    log(f"bench: headline {value:.2f} images/s, iterations {head['iters'][-1]}, "
        f"bf16 part {head['iters_low'][-1]}")

    fp32 = None
    if not args.no_fp32:
        log("bench: fp32-plain arm")
        fp32 = time_arm(torch, ctx, y, args.steps, args.warmup, conv_prec="f32", **common)
        fp32["value"] = n_img * len(fp32["step_s"]) / fp32["total_s"]
        log(f"bench: fp32 plain {fp32['value']:.2f} images/s, iterations {fp32['iters'][-1]}")

    # rooflines of the 64->64 conv kernels of the timed solves; the dominant one
    # (by device time) is `roofline`, the other `roofline_other`
    def conv_roofline(cls):
        ms, launches, px = head["prof"][cls]
        if not launches:
            return None
        split = cls == "conv64_bf16x3"
        avg_ms = ms / launches
        flops_per_launch = FLOP_PER_PX_64 * px / launches
        achieved = flops_per_launch / (avg_ms * 1e-3)
        # the conv's own (algorithmic) flops against the dense bf16 matrix-core
        # peak; split-bf16 issues three bf16 products per term, so it can reach at
        # most a third of that peak, reported separately
        peak = BF16_PEAK
        tr = TRAFFIC[cls]
        # bytes per pixel of an E_ACT pass (in + out) and an E_DELTA pass
        # (in + sigma operand + out), which the solve runs in equal numbers
        per_px = (512.0 + 768.0) / 2 if split else (256.0 + 384.0) / 2
        return {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": (tr["bytes_per_px"] * px / launches
                            if sources_sha256(tr["sources"]) == tr["sha256"] else None),
                "traffic_unit": "bytes per launch",
                "algorithmic_bytes": per_px * px / launches,
                "kernel": ("conv_halves_kernel<bf16x3, 64>" if split
                           else "conv_halves_kernel<bf16, 64>"),
                "launches": launches, "sampled_every": args.sample_every,
                "matrix_core_products_per_flop": 3 if split else 1,
                "frac_of_product_ceiling": achieved / (peak / (3.0 if split else 1.0)),
                "avg_launch_us": avg_ms * 1e3,
                "total_ms": ms, "flop_per_launch": flops_per_launch}
    rl = {c: conv_roofline(c) for c in ("conv64_bf16x3", "conv64_bf16")}
    order = sorted((r for r in rl.values() if r), key=lambda r: -r["total_ms"])
    roofline = order[0]
    roofline_other = order[1] if len(order) > 1 else None
    phases = class_breakdown(torch, ctx, y, **head_kw)

    also = None if args.no_also else also_measured(torch, args.poll, ws, ctx, y, tau)
    if also is not None and not args.no_paper_workloads:
        also.update(paper_workloads(torch, args.poll))

    cpu = None
    if not args.no_cpu_baseline:
        ref_iters = float(np.mean(fp32["iters"][-1])) if fp32 else float(np.mean(head["iters"][-1]))
        log("bench: cpu baseline (float64 oracle on the host)")
        cpu = cpu_baseline(ref_iters)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * head["total_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+bf16x3+f32" if args.refine == "bf16x3" else "bf16+f32",
        "data": "synthetic",
        "config": {
            "workload": "i-DEQ deblurring, 8x3x256x256, circular 9x9 gaussian (sigma 1.6), "
                        "noise 0.01, 5-layer 64-channel softplus regularizer, rel. residual 1e-4",
            "arm": ("bf16 convs, then split-bf16 (hi/lo, 3 products) convs to rel 1e-4, then "
                    "fp32 convs until an fp32 update has rel < 1e-4" if args.refine == "bf16x3"
                    else "bf16 convs, then fp32 convs to rel 1e-4") + f"; init={init}",
            "arithmetic": "conv operands bf16 (fp32 accumulate), then split-bf16 (each fp32 "
                          "operand as bf16 hi + lo, 3 products, fp32 accumulate), then fp32; "
                          "state tensors fp32; per-image residuals, stopping test and "
                          "reductions fp64",
            "updates_per_image_by_arithmetic": {
                "bf16": head["iters_low"][-1], "bf16x3": head["iters_mid"][-1],
                "f32": [a - b - c for a, b, c in zip(head["iters"][-1], head["iters_low"][-1],
                                                     head["iters_mid"][-1])]},
            "global_batch": n_img,
            "parallelism": "single GPU",
        },
        "iters_per_image": head["iters"][-1],
        "bf16_iters_per_image": head["iters_low"][-1],
        "split_iters_per_image": head["iters_mid"][-1],
        "fp32_plain": None if fp32 is None else {
            "value": fp32["value"], "iters_per_image": fp32["iters"][-1],
            "ms_per_step": 1e3 * fp32["total_s"] / len(fp32["step_s"])},
        "speedup_vs_fp32_plain": None if fp32 is None else value / fp32["value"],
        "step_size": {"L": L, "tau": tau, "power_iteration_ms": t_L * 1e3},
        "device_ms_by_class_one_solve": phases,
        "roofline": roofline,
        "roofline_other": roofline_other,
        "also_measured": also,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
