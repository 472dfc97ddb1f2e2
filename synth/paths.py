"""Light-path records from a counter-based generator.

Record layout (the input format of both shading forms):

* paths are pixel-major: pixel q owns paths [q*spp, (q+1)*spp);
* ``hdr[p]`` (uint32): light id in bits 0-23, path length L_p (number of
  reflectance vertices, 0-255) in bits 24-31;
* ``pix_first[q]`` (uint32): index of pixel q's first vertex record; a
  pixel's paths store their vertices back to back, in path order;
* ``vtx[j]`` (2 x uint32): texel/material index, then the IEEE-754 bits of
  the float32 vertex weight.

The random draws come from a counter-based generator so that any path can be
produced on its own (the GPU generator and the sampled-pixel checks rely on
this).  It is SplitMix64's output function (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
``key + (counter + 1) * 0x9E3779B97F4A7C15`` (mod 2^64):

* stream key      = mix64(mix64(seed) + stream)   (stream 1: paths, 2: vertices)
* path p          : r = rand64(key_path, p)
  L_p   = l_min + ((r & 0xFFFFFFFF) * (l_max - l_min + 1)) >> 32
  light = ((r >> 32) * n_illum) >> 32
* vertex v of p   : r = rand64(key_vtx, p * 256 + v)
  texel  = ((r & 0xFFFFFFFF) * n_tex) >> 32
  weight = (r >> 40) * 2^-24            (exact float32 in [0, 1))
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_LO32 = np.uint64(0xFFFFFFFF)
STREAM_PATH = 1
STREAM_VERTEX = 2
STREAM_INDEX = 3


def mix64(z):
    """SplitMix64 output function on uint64 (arrays or scalars), wrapping mod 2^64."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        return np.uint64(mix64(mix64(np.uint64(seed)) + np.uint64(stream)))


def rand64(key, ctr):
    ctr = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(key) + (ctr + np.uint64(1)) * GOLDEN)


def _range32(r, n):
    """Map the low 32 bits of r to [0, n) by multiply-shift."""
    return ((r & _LO32) * np.uint64(n)) >> np.uint64(32)


@dataclass(frozen=True)
class PathSpec:
    """A frame's path population."""
    n_pixels: int
    spp: int
    l_min: int
    l_max: int
    n_tex: int
    n_illum: int
    seed: int

    @property
    def n_paths(self) -> int:
        return self.n_pixels * self.spp


def path_headers(spec: PathSpec, p: np.ndarray):
    """(L, light id) of the given global path indices."""
    r = rand64(stream_key(spec.seed, STREAM_PATH), p)
    nl = spec.l_max - spec.l_min + 1
    length = (np.uint64(spec.l_min) + _range32(r, nl)).astype(np.int64)
    light = ((r >> np.uint64(32)) * np.uint64(spec.n_illum)) >> np.uint64(32)
    return length, light.astype(np.int64)


def vertex_draws(spec: PathSpec, p: np.ndarray, v: np.ndarray):
    """(texel, weight) of vertex v of path p, elementwise over the arrays."""
    ctr = np.asarray(p, dtype=np.uint64) * np.uint64(256) + np.asarray(v, dtype=np.uint64)
    r = rand64(stream_key(spec.seed, STREAM_VERTEX), ctr)
    texel = _range32(r, spec.n_tex).astype(np.uint32)
    weight = ((r >> np.uint64(40)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
    return texel, weight


def gen_paths(spec: PathSpec, chunk_pixels: int = 1 << 20):
    """Whole-frame records: (hdr uint32[P], pix_first uint32[n_pixels], vtx uint32[V, 2])."""
    if not (0 <= spec.l_min <= spec.l_max <= 255):
        raise ValueError("path lengths must satisfy 0 <= l_min <= l_max <= 255")
    if not (1 <= spec.n_illum <= 1 << 24):
        raise ValueError("light count must be in [1, 2^24]")
    hdr = np.empty(spec.n_paths, dtype=np.uint32)
    lengths = np.empty(spec.n_paths, dtype=np.int64)
    for q0 in range(0, spec.n_pixels, chunk_pixels):
        q1 = min(spec.n_pixels, q0 + chunk_pixels)
        p = np.arange(q0 * spec.spp, q1 * spec.spp, dtype=np.uint64)
        length, light = path_headers(spec, p)
        lengths[q0 * spec.spp:q1 * spec.spp] = length
        hdr[q0 * spec.spp:q1 * spec.spp] = (light | (length << 24)).astype(np.uint32)
    per_pixel = lengths.reshape(spec.n_pixels, spec.spp).sum(axis=1)
    total = int(per_pixel.sum())
    if total >= 1 << 32:
        raise ValueError("more than 2^32 - 1 vertex records in one frame")
    pix_first = np.zeros(spec.n_pixels, dtype=np.uint32)
    if spec.n_pixels > 1:
        pix_first[1:] = np.cumsum(per_pixel[:-1]).astype(np.uint32)
    vtx = np.empty((total, 2), dtype=np.uint32)
    path_first = np.zeros(spec.n_paths + 1, dtype=np.int64)
    np.cumsum(lengths, out=path_first[1:])
    step = chunk_pixels * spec.spp
    for p0 in range(0, spec.n_paths, step):
        p1 = min(spec.n_paths, p0 + step)
        ls = lengths[p0:p1]
        j0, j1 = path_first[p0], path_first[p1]
        pid = np.repeat(np.arange(p0, p1, dtype=np.int64), ls)
        v = np.arange(j1 - j0, dtype=np.int64) - np.repeat(path_first[p0:p1] - j0, ls)
        texel, weight = vertex_draws(spec, pid, v)
        vtx[j0:j1, 0] = texel
        vtx[j0:j1, 1] = weight.view(np.uint32)
    return hdr, pix_first, vtx


def path_records(spec: PathSpec, paths: np.ndarray):
    """Records of selected paths, without generating the frame.

    Returns (L int64[P], light int64[P], texel int64[P, Lmax], weight
    float32[P, Lmax]); entries past a path's length are 0.
    """
    p = np.asarray(paths, dtype=np.uint64)
    length, light = path_headers(spec, p)
    lmax = max(1, int(length.max()) if length.size else 1)
    v = np.arange(lmax, dtype=np.uint64)
    texel, weight = vertex_draws(spec, p[:, None], v[None, :])
    live = v[None, :].astype(np.int64) < length[:, None]
    return (length, light, np.where(live, texel, 0).astype(np.int64),
            np.where(live, weight, np.float32(0)).astype(np.float32))


def records_of_pixels(spec: PathSpec, pixels):
    """Record arrays (hdr, pix_first, vtx) of a subset of a frame's pixels,
    in the frame's layout, drawn without generating the whole frame."""
    pixels = np.asarray(pixels, dtype=np.int64)
    paths = (pixels[:, None] * spec.spp + np.arange(spec.spp)[None, :]).ravel()
    length, light, tex, wt = path_records(spec, paths)
    hdr = (light | (length << 24)).astype(np.uint32)
    per_px = length.reshape(-1, spec.spp).sum(axis=1)
    pf = np.zeros(pixels.size, dtype=np.uint32)
    if pixels.size > 1:
        pf[1:] = np.cumsum(per_px[:-1])
    live = np.arange(tex.shape[1])[None, :] < length[:, None]
    vtx = np.stack([tex[live].astype(np.uint32), wt[live].view(np.uint32)], axis=1)
    return hdr, pf, vtx


def chain_records(n_chains: int, bounces: int):
    """Records of the multi-bounce chains: one pixel per (bounce b, chain c)
    for b = 0 .. bounces, pixel b * n_chains + c, one sample whose path
    starts at light c and meets b reflectances, texels c * bounces + v for
    v < b, all weights 1 (b = 0 is the light seen directly).  Returns
    (hdr uint32, pix_first uint32, vtx uint32 [V, 2]) in the frame layout."""
    c = np.arange(n_chains, dtype=np.int64)
    b = np.arange(bounces + 1, dtype=np.int64)
    length = np.repeat(b, n_chains)
    light = np.tile(c, bounces + 1)
    hdr = (light | (length << 24)).astype(np.uint32)
    pf = np.zeros(length.size, dtype=np.uint32)
    pf[1:] = np.cumsum(length[:-1])
    tex = np.concatenate([(c[:, None] * bounces + np.arange(bb)[None, :]).ravel() for bb in b])
    vtx = np.stack([tex.astype(np.uint32),
                    np.full(tex.size, np.float32(1.0)).view(np.uint32)], axis=1)
    return hdr, pf, vtx


def uniform_indices(seed: int, ctr0: int, count: int, n: int) -> np.ndarray:
    """count indices uniform in [0, n) drawn at counters ctr0 .. ctr0+count-1."""
    r = rand64(stream_key(seed, STREAM_INDEX), np.arange(ctr0, ctr0 + count, dtype=np.uint64))
    return _range32(r, n).astype(np.uint32)
