"""Spectral textures: Perlin-noise-weighted blends of basis spectra."""

from __future__ import annotations

import numpy as np

# 8 unit-ish gradient directions for 2-D gradient noise.
_GRADS = np.array([[1, 1], [-1, 1], [1, -1], [-1, -1],
                   [1, 0], [-1, 0], [0, 1], [0, -1]], dtype=np.float64)


def _fade(t):
    # Quintic interpolant of Perlin's improved noise (SIGGRAPH 2002).
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _noise2(perm: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Improved-Perlin-style 2-D gradient noise with a 256-entry permutation."""
    xi = np.floor(x).astype(np.int64)
    yi = np.floor(y).astype(np.int64)
    xf = x - xi
    yf = y - yi
    xi &= 255
    yi &= 255
    u = _fade(xf)
    v = _fade(yf)

    def corner(dx, dy):
        h = perm[perm[(xi + dx) & 255] + ((yi + dy) & 255)] & 7
        g = _GRADS[h]
        return g[..., 0] * (xf - dx) + g[..., 1] * (yf - dy)

    n00 = corner(0, 0)
    n10 = corner(1, 0)
    n01 = corner(0, 1)
    n11 = corner(1, 1)
    nx0 = n00 + u * (n10 - n00)
    nx1 = n01 + u * (n11 - n01)
    return nx0 + v * (nx1 - nx0)


def perlin_weights(seed: int, side: int, n_fields: int = 16, cells: int = 8,
                   sharpness: float = 4.0, rows: slice | None = None) -> np.ndarray:
    """Per-texel blend weights, softmax over fields of sharpness * noise_j.

    Field j uses its own permutation (seeded by (seed, j)); `cells` lattice
    cells span the texture.  Returns (texels, n_fields) float64 for the
    requested row range (all rows by default), texel index = row * side + col.
    """
    rows = rows or slice(0, side)
    r0, r1 = rows.start, rows.stop
    yy, xx = np.meshgrid(np.arange(r0, r1, dtype=np.float64),
                         np.arange(side, dtype=np.float64), indexing="ij")
    x = (xx + 0.5) * (cells / side)
    y = (yy + 0.5) * (cells / side)
    logits = np.empty((x.size, n_fields))
    for j in range(n_fields):
        perm = np.random.default_rng([seed, j]).permutation(256)
        perm = np.concatenate([perm, perm]).astype(np.int64)
        logits[:, j] = sharpness * _noise2(perm, x, y).ravel()
    logits -= logits.max(axis=1, keepdims=True)
    w = np.exp(logits)
    w /= w.sum(axis=1, keepdims=True)
    return w


def perlin_texture(seed: int, side: int, basis: np.ndarray, ld: int | None = None,
                   chunk_rows: int = 256, base: int | None = None) -> np.ndarray:
    """side x side spectral texture: texel = sum_j weight_j * basis_j.

    `basis` is (n_fields, n) with entries in [0, 1]; the weights sum to 1, so
    texels stay in [0, 1].  With `base` (dividing side), the weight field is
    computed on a base x base grid and each weight covers a block of
    (side/base)^2 texels, which keeps very large textures cheap to build.
    Returns (side*side, ld) float32 with columns [n, ld) zero (ld defaults to n).
    """
    nf, n = basis.shape
    ld = n if ld is None else ld
    out = np.zeros((side * side, ld), dtype=np.float32)
    b64 = basis.astype(np.float64)
    if base is not None and base < side:
        f = side // base
        w = perlin_weights(seed, base, nf)            # (base*base, nf)
        blended = (w @ b64).astype(np.float32).reshape(base, base, n)
        for r0 in range(0, side, chunk_rows):
            r1 = min(side, r0 + chunk_rows)
            rows = blended[np.arange(r0, r1) // f]     # (r1-r0, base, n)
            out[r0 * side:r1 * side, :n] = np.repeat(rows, f, axis=1).reshape(-1, n)
        return out
    for r0 in range(0, side, chunk_rows):
        r1 = min(side, r0 + chunk_rows)
        w = perlin_weights(seed, side, nf, rows=slice(r0, r1))
        out[r0 * side:r1 * side, :n] = (w @ b64).astype(np.float32)
    return out
