"""The five synthetic workloads (shapes and distributions of the paper's use).

Their parameters live in ``configs/cfg{c}.json`` (see ``config``); this module
builds the inputs.  Seeds: every random draw for workload c and purpose j
comes from ``numpy.random.default_rng([c, j])`` with j = 0 spectra tables,
1 texture, 3 codec, 4 codec-fit pools, 5 serving arrivals, 6 multi-bounce
chains; the counter-based path generator takes the configuration's
``path_seed`` (1000 c + 2).

* c = 0  tiny parity case: n = 31, k = 6, random U[0,1] codec, 64
  reflectances, 8 lights (4 Planck, 4 narrow-band), 256 x 256 px, 1 spp,
  one reflectance vertex per path.
* c = 1  frame scale: 1920 x 1080 px, 16 spp, L in 1..4, 1024^2 x 31
  Perlin-blended texture of 16 basis reflectances, 32 lights (16 + 16).
* c = 2  codec fit: pools of reflectances and lights (half Planck, half
  narrow-band) at n in {31, 81}; held-out chains for the multi-bounce
  evaluation (purpose 6).
* c = 3  serving: request stream (see the serving module).
* c = 4  stress: n = 81, k = 9, 3840 x 2160 px, 64 spp, L in 1..8,
  4096^2 x 81 texture (Perlin weights on a 512^2 grid, one weight per 8x8
  texel block), 256 lights (64 Planck, 192 narrow-band sigma 5-10).
"""

from __future__ import annotations

import numpy as np

from .config import config
from .paths import PathSpec
from .spectra import (cmf_matrix, codec_uniform, illuminant_table, reflectances,
                      wavelengths)
from .texture import perlin_texture


def _rng(c: int, j: int) -> np.random.Generator:
    return np.random.default_rng([c, j])


def workload(c: int, *, width: int | None = None, height: int | None = None,
             spp: int | None = None, texture_side: int | None = None,
             k: int | None = None, ld_tex: int | None = None) -> dict:
    """Inputs of workload c.  Keyword overrides shrink a workload for tests.

    Returns a dict with: n, k, lam, T (3 x n), refl (texels x ld_tex,
    float32), n_tex, illum (n_illum x n), E (k x n), D (n x k), paths
    (PathSpec), width, height.
    """
    if c not in (0, 1, 4):
        raise ValueError(f"workload {c} has no frame inputs")
    cfg = config(c)
    n, kk = cfg["n"], cfg["k"]
    t0 = _rng(c, 0)
    lt = cfg["lights"]
    if c == 0:
        refl = reflectances(t0, n, cfg["reflectances"])
        illum = illuminant_table(t0, n, lt["planck"], lt["narrow"], *lt["narrow_sigma_nm"])
    else:
        tx = cfg["texture"]
        basis = reflectances(t0, n, tx["basis"])
        illum = illuminant_table(t0, n, lt["planck"], lt["narrow"], *lt["narrow_sigma_nm"])
        side = texture_side or tx["side"]
        base = min(side, tx["perlin_side"]) if "perlin_side" in tx else None
        refl = perlin_texture(tx["perlin_seed"], side, basis, ld=ld_tex, base=base)
    fr = cfg["frame"]
    w, h, s = fr["width"], fr["height"], fr["spp"]
    lmin, lmax = fr["path_length"]
    if ld_tex is not None and c == 0:
        pad = np.zeros((refl.shape[0], ld_tex), dtype=np.float32)
        pad[:, :n] = refl
        refl = pad
    kk = k or kk
    e, d = codec_uniform(_rng(c, 3), kk, n)
    w, h, s = width or w, height or h, spp or s
    spec = PathSpec(n_pixels=w * h, spp=s, l_min=lmin, l_max=lmax,
                    n_tex=refl.shape[0], n_illum=illum.shape[0], seed=cfg["path_seed"])
    return dict(n=n, k=kk, lam=wavelengths(n), T=cmf_matrix(n), refl=refl,
                n_tex=refl.shape[0], illum=illum, E=e, D=d, paths=spec,
                width=w, height=h)


def codec_pools(n: int, count: int, seed_c: int = 2):
    """Reflectance and light pools for codec fitting (config-0 generators;
    lights half Planckian, half narrow-band).  Returns two (count, n) float32."""
    rng = _rng(seed_c, 4)
    refl = reflectances(rng, n, count)
    sigma = config(2)["lights"]["narrow_sigma_nm"]
    illum = illuminant_table(rng, n, count // 2, count - count // 2, *sigma)
    return refl, illum


def bounce_chains(n: int, count: int, bounces: int = 3):
    """Held-out spectra of the multi-bounce evaluation: `count` lights (half
    Planckian, half narrow-band) and bounces reflectances per chain, drawn
    from the codec-fit generators with their own seed.  Returns
    (refl (count * bounces, n) with chain c's reflectances in rows
    c * bounces .. c * bounces + bounces - 1, lights (count, n)), float32."""
    rng = _rng(2, 6)
    refl = reflectances(rng, n, count * bounces)
    sigma = config(2)["lights"]["narrow_sigma_nm"]
    lights = illuminant_table(rng, n, count // 2, count - count // 2, *sigma)
    return refl, lights
