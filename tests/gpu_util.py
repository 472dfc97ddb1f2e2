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
