"""Reader of the light-path record format (oracle side).

Format: pixel q owns paths [q*spp, (q+1)*spp); hdr[p] holds the light id in
bits 0-23 and the path length L_p in bits 24-31; pix_first[q] is the index of
pixel q's first vertex record and the pixel's paths store their vertices back
to back in path order; vtx[j] = (texel index, float32 weight bits).
"""

from __future__ import annotations

import numpy as np


def unpack(hdr, pix_first, vtx, spp: int):
    """Per-path (L, light, first vertex index) and per-vertex (texel, weight).

    Returns L int64[P], light int64[P], first int64[P], texel int64[V],
    weight float64[V].
    """
    hdr = np.asarray(hdr, dtype=np.uint32)
    length = (hdr >> 24).astype(np.int64)
    light = (hdr & 0xFFFFFF).astype(np.int64)
    n_pixels = hdr.size // spp
    lp = length.reshape(n_pixels, spp)
    # exclusive prefix of L inside each pixel, plus the pixel's first record
    within = np.cumsum(lp, axis=1) - lp
    first = (np.asarray(pix_first, dtype=np.int64)[:, None] + within).ravel()
    vtx = np.asarray(vtx, dtype=np.uint32).reshape(-1, 2)
    texel = vtx[:, 0].astype(np.int64)
    weight = vtx[:, 1].view(np.float32).astype(np.float64)
    return length, light, first, texel, weight


def check(hdr, pix_first, vtx, spp: int, n_tex: int, n_illum: int):
    """Counts of invalid records: (bad lights, bad texels, bad pixel ranges).

    A pixel range is bad when its records would run past the vertex array;
    texels are only examined inside good ranges.
    """
    length, light, first, texel, _ = unpack(hdr, pix_first, vtx, spp)
    n_v = texel.size
    bad_light = int(np.count_nonzero(light >= n_illum))
    n_pixels = length.size // spp
    end = np.asarray(pix_first, dtype=np.int64) + length.reshape(n_pixels, spp).sum(axis=1)
    good_px = end <= n_v
    bad_range = int(np.count_nonzero(~good_px))
    # each vertex counts once per good pixel range that covers it
    cover = np.zeros(n_v + 1, dtype=np.int64)
    np.add.at(cover, np.asarray(pix_first, dtype=np.int64)[good_px], 1)
    np.add.at(cover, end[good_px], -1)
    times = np.cumsum(cover)[:n_v]
    bad_tex = int(times[texel >= n_tex].sum())
    return bad_light, bad_tex, bad_range
