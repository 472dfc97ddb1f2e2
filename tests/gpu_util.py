"""Helpers shared by the GPU tests (test-side packing of synthetic inputs)."""

import numpy as np
import torch

import synth
from synth import records_of_pixels  # noqa: F401


def dev_f32(a, ld=None):
    """numpy (m, n) -> device float32 with rows padded to ld (multiple of 4)."""
    a = np.asarray(a, dtype=np.float32)
    m, n = a.shape
    ld = ld or 4 * ((n + 3) // 4)
    out = np.zeros((m, ld), dtype=np.float32)
    out[:, :n] = a
    return torch.from_numpy(out).cuda()


def to_np(t):
    return t.detach().cpu().numpy()


def box_codec(k, n, beta=10.0, floor=1e-3):
    """Pre-softplus weights (k x n, n x k) of a box-filter codec: code j
    averages the samples of the j-th of k equal bins and the decoder holds
    each bin's average, every other weight being `floor` after the softplus
    (Eq. 5 inverted).  For the synthetic spectra this is a near fit (the
    Eq. 8 loss some 4,000 times below that of the random initial weights at
    n = 81, k = 9), where gradients are differences of nearly equal terms."""
    edges = np.linspace(0, n, k + 1).round().astype(int)
    E = np.full((k, n), floor)
    D = np.full((n, k), floor)
    for j in range(k):
        lo, hi = edges[j], edges[j + 1]
        E[j, lo:hi] = 1.0 / (hi - lo)
        D[lo:hi, j] = 1.0
    inv = lambda y: np.log(np.expm1(beta * y)) / beta
    return inv(E), inv(D)
