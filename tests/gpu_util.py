"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np
import torch

import synth


def dev():
    return torch.device("cuda:0")


def to_gpu(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def to_np(t):
    return t.detach().cpu().double().numpy()


def rel_err(a, b):
    """max over images of ||a - b|| / ||b||."""
    d = np.sqrt(np.sum((a - b) ** 2, axis=(1, 2, 3)))
    r = np.sqrt(np.sum(b ** 2, axis=(1, 2, 3)))
    return float(np.max(d / r))


def net_layers(name, seed=0, bias_seed=None):
    return synth.he_normal_net(synth.net_channels(name), seed, bias_seed=bias_seed)
