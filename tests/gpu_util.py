"""Helpers shared by the GPU tests (test-side packing of synthetic inputs)."""

import numpy as np
import torch

import synth


def dev_f32(a, ld=None):
    """numpy (m, n) -> device float32 with rows padded to ld (multiple of 4)."""
    a = np.asarray(a, dtype=np.float32)
    m, n = a.shape
    ld = ld or 4 * ((n + 3) // 4)
    out = np.zeros((m, ld), dtype=np.float32)
    out[:, :n] = a
    return torch.from_numpy(out).cuda()


def records_of_pixels(spec: synth.PathSpec, pixels: np.ndarray):
    """Record arrays (synth layout) of a subset of a frame's pixels, built from
    the counter-based generator without generating the frame."""
    pixels = np.asarray(pixels, dtype=np.int64)
    paths = (pixels[:, None] * spec.spp + np.arange(spec.spp)[None, :]).ravel()
    L, light, tex, wt = synth.path_records(spec, paths)
    hdr = (light | (L << 24)).astype(np.uint32)
    per_px = L.reshape(-1, spec.spp).sum(axis=1)
    pf = np.zeros(pixels.size, dtype=np.uint32)
    pf[1:] = np.cumsum(per_px[:-1])
    live = np.arange(tex.shape[1])[None, :] < L[:, None]
    vtx = np.stack([tex[live].astype(np.uint32), wt[live].view(np.uint32)], axis=1)
    return hdr, pf, vtx


def to_np(t):
    return t.detach().cpu().numpy()
