"""Writes tests/golden/headline_image0_reference.npz from the float64 oracle only.

Image 0 of the headline deblurring batch (generator id 2, 3 x 256 x 256,
circular 9x9 Gaussian blur sigma 1.6, noise 0.01, the 5-layer 64-channel
SoftPlus regularizer from seed 0, lambda 1, beta 0.5), with a fixed step size
tau = 0.16 (below 2 / L for L ~ 5.3 of this problem):
  * ws_x0      the learned warm start x0 = y + W_phi(y) of the packaged weights
               (oracle.warmstart.forward, float64);
  * x_ws_10    10 i-DEQ updates (Alg. 1) from ws_x0;
  * x_y_30     30 i-DEQ updates from x0 = y.
Stored as float32 (their rounding, 6e-8 relative, is far below the tests'
tolerances).  The oracle takes several seconds per iteration of a 256^2 image
on a few host cores, so the run takes tens of minutes; the fixed point itself
(relative step 1e-9) is out of reach: the iteration contracts by about 0.999
per step late in the solve.

Usage: python tests/golden/make_headline_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import operators as O, regularizer as R, solver as S, warmstart as WS  # noqa: E402

TAU = 0.16


def main():
    t0 = time.time()
    layers = synth.he_normal_net(synth.net_channels("rgb64"), 0)
    op = O.Operator("blur", synth.gaussian_taps(9, 1.6))
    xt, nz = synth.make_batch(2, 1, 3, 256, 256)
    y = op.A(xt) + 0.01 * nz
    P = S.Problem(op, R.Net(layers), 1.0)
    flat = np.load(os.path.join(ROOT, "paper_2605_19705_amd", "weights", "warmstart_deblur.npy"))
    wl, o = [], 0
    for cin, cout in synth.warmstart_channels():
        nw = cout * cin * 9
        wl.append((flat[o:o + nw].reshape(cout, cin, 3, 3), flat[o + nw:o + nw + cout]))
        o += nw + cout
    assert o == flat.size
    x0, _ = WS.forward(wl, y)
    print(f"warm start done ({time.time() - t0:.0f} s)", flush=True)
    x10, _ = S.ideq_solve(P, y, x0, 0.5, TAU, fixed_iters=10)
    print(f"10 updates from the warm start done ({time.time() - t0:.0f} s)", flush=True)
    x30, _ = S.ideq_solve(P, y, y, 0.5, TAU, fixed_iters=30)
    print(f"30 updates from y done ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "headline_image0_reference.npz"), tau=TAU,
                        ws_x0=x0.astype(np.float32), x_ws_10=x10.astype(np.float32),
                        x_y_30=x30.astype(np.float32))


if __name__ == "__main__":
    main()
