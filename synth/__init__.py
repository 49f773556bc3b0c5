"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module only *draws* data: ground-truth images, unit-variance noise fields,
He-normal conv weights and the blur taps that define the forward operator.
It contains none of the restoration method's arithmetic (no operator is
applied here; the measurement y = A(x) + sigma * n is formed by whichever side
consumes these arrays).

Everything is float64 NumPy, drawn from ``numpy.random.default_rng`` with the
seeds documented on each function, so both sides see bit-identical inputs.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "ground_truth", "noise_field", "make_batch", "he_normal_net",
    "gaussian_taps", "uniform_taps", "net_channels", "warmstart_channels",
    "random_field", "warmstart_init", "pixel_mask", "cartesian_mask",
]


def ground_truth(cfg_id: int, img_idx: int, c: int, h: int, w: int) -> np.ndarray:
    """Piecewise-constant plus smooth test image in [0, 1], shape (c, h, w).

    Recipe (per image, ``rng = default_rng([cfg_id, img_idx])``):
      * 6 axis-aligned rectangles, top-left corner uniform over the image,
        integer side lengths uniform in [h//8, h//2] (resp. w), clipped at the
        border, painted in draw order with a per-channel colour ~ U[0, 1];
      * 4 isotropic Gaussian blobs, centre ~ U[0,h) x U[0,w), std ~ U[2, 6] px,
        per-channel amplitude ~ U[0.3, 1], added;
      * clip to [0, 1].
    The same ``rng`` then continues with :func:`noise_field` draws, so call
    :func:`make_batch` to get the pair consistently.
    """
    rng = np.random.default_rng([cfg_id, img_idx])
    return _draw_image(rng, c, h, w)


def _draw_image(rng, c, h, w):
    img = np.zeros((c, h, w), dtype=np.float64)
    for _ in range(6):
        y0 = int(rng.integers(0, h))
        x0 = int(rng.integers(0, w))
        hh = int(rng.integers(max(1, h // 8), max(1, h // 2) + 1))
        ww = int(rng.integers(max(1, w // 8), max(1, w // 2) + 1))
        col = rng.uniform(0.0, 1.0, size=c)
        img[:, y0:y0 + hh, x0:x0 + ww] = col[:, None, None]
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64),
                         np.arange(w, dtype=np.float64), indexing="ij")
    for _ in range(4):
        cy = rng.uniform(0.0, h)
        cx = rng.uniform(0.0, w)
        s = rng.uniform(2.0, 6.0)
        amp = rng.uniform(0.3, 1.0, size=c)
        blob = np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * s * s))
        img += amp[:, None, None] * blob[None]
    return np.clip(img, 0.0, 1.0)


def noise_field(cfg_id: int, img_idx: int, c: int, h: int, w: int) -> np.ndarray:
    """Standard-normal field (c, h, w) drawn right after the image's own draws."""
    rng = np.random.default_rng([cfg_id, img_idx])
    _draw_image(rng, c, h, w)
    return rng.standard_normal((c, h, w))


def make_batch(cfg_id: int, n: int, c: int, h: int, w: int, first: int = 0):
    """(x_true, noise) each of shape (n, c, h, w), images ``first..first+n-1``."""
    xs = np.empty((n, c, h, w))
    ns = np.empty((n, c, h, w))
    for i in range(n):
        rng = np.random.default_rng([cfg_id, first + i])
        xs[i] = _draw_image(rng, c, h, w)
        ns[i] = rng.standard_normal((c, h, w))
    return xs, ns


def random_field(seed, shape) -> np.ndarray:
    """Plain standard-normal array from ``default_rng(seed)`` (test vectors,
    power-iteration start vectors, loss targets)."""
    return np.random.default_rng(seed).standard_normal(shape)


def net_channels(name: str):
    """Channel lists of the regularizer networks N_theta used by the workloads."""
    if name == "gray16":      # 3-layer 1->16->16->1
        return [1, 16, 16, 1]
    if name == "rgb64":       # 5-layer 3->64->64->64->64->3
        return [3, 64, 64, 64, 64, 3]
    raise ValueError(name)


def he_normal_net(channels, seed: int = 0, bias_seed=None):
    """He-normal 3x3 conv weights, layer by layer from ``default_rng(seed)``.

    Layer l has W_l ~ N(0, 2 / (9 * C_in)) with shape (C_out, C_in, 3, 3) drawn
    as ``rng.standard_normal`` in C order; biases are zero unless ``bias_seed``
    is given (then N(0, 0.1^2) from ``default_rng(bias_seed)``, used by tests to
    exercise the bias path).
    Returns a list of (W, b) float64 pairs.
    """
    rng = np.random.default_rng(seed)
    brng = None if bias_seed is None else np.random.default_rng(bias_seed)
    out = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        W = rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9.0 * cin))
        b = np.zeros(cout) if brng is None else 0.1 * brng.standard_normal(cout)
        out.append((W, b))
    return out


def gaussian_taps(size: int = 9, sigma: float = 1.6) -> np.ndarray:
    """Normalised isotropic Gaussian blur taps (size x size), centred."""
    r = (size - 1) / 2.0
    t = np.arange(size, dtype=np.float64) - r
    g = np.exp(-(t[:, None] ** 2 + t[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def uniform_taps(size: int = 7) -> np.ndarray:
    """Uniform (box) blur taps, size x size, summing to one."""
    return np.full((size, size), 1.0 / (size * size))


def warmstart_channels():
    """Layer plan of the warm-start encoder-decoder (see the package docs):
    enc1: 3->32->32 (full res), 2x2 average pool, enc2: 32->64->64->64->64
    (half res), nearest upsample, concat with enc1 output (64+32=96),
    dec: 96->32->32->3. Returned as (c_in, c_out) per conv in execution order."""
    return [(3, 32), (32, 32), (32, 64), (64, 64), (64, 64), (64, 64),
            (96, 32), (32, 32), (32, 3)]


def warmstart_init(seed: int = 0, out_scale: float = 0.1):
    """Initial weights of the warm-start encoder-decoder: He-normal
    W ~ N(0, 2 / (9 * C_in)) drawn layer by layer from ``default_rng(seed)``
    in C order, the output layer scaled by ``out_scale`` (so that the initial
    network output is small and x0 starts close to y), zero biases."""
    rng = np.random.default_rng(seed)
    chans = warmstart_channels()
    out = []
    for i, (cin, cout) in enumerate(chans):
        W = rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9.0 * cin))
        if i == len(chans) - 1:
            W = W * out_scale
        out.append((W, np.zeros(cout)))
    return out


def pixel_mask(seed, h: int, w: int, keep: float = 0.5) -> np.ndarray:
    """Inpainting mask (h, w) of 0.0 / 1.0: each pixel is kept (1) independently
    with probability ``keep``, from ``default_rng(seed).random((h, w)) < keep``.
    A removed pixel loses all of its channels."""
    return (np.random.default_rng(seed).random((h, w)) < keep).astype(np.float64)


def cartesian_mask(seed, h: int, w: int, accel: int = 8, center_lines: int = None) -> np.ndarray:
    """Cartesian k-space sampling mask (h, w) of 0.0 / 1.0 in the FFT's own
    index order (frequency 0 at index 0): whole lines of fixed row frequency
    ky are sampled, every column kx of a sampled line.

    h // accel lines are sampled in total: the ``center_lines`` lowest
    frequencies (default max(2, round(0.04 h)), the rows with |ky| smallest,
    ky = 0 first) and then lines drawn uniformly without replacement from the
    others by ``default_rng(seed).choice``.
    """
    n_lines = max(1, h // accel)
    if center_lines is None:
        center_lines = max(2, int(round(0.04 * h)))
    center_lines = min(center_lines, n_lines)
    freq = np.fft.fftfreq(h) * h                # signed row frequency of each index
    order = np.argsort(np.abs(freq), kind="stable")
    chosen = list(order[:center_lines])
    rest = np.setdiff1d(np.arange(h), chosen)
    extra = np.random.default_rng(seed).choice(rest, size=n_lines - center_lines, replace=False)
    rows = np.zeros(h, dtype=np.float64)
    rows[chosen] = 1.0
    rows[extra] = 1.0
    return np.repeat(rows[:, None], w, axis=1)
