"""Multi-bounce evaluation of a codec (Eq. 10, Sec. 4.5) on the GPU.

A chain is a light L and reflectances R_1, R_2, ... met in turn; after b
bounces the radiance is S_b = R_b * S_{b-1}, S_0 = L.  The chains are laid
out as a one-sample frame, pixel b * C + c holding chain c after b bounces
(b = 0 is the light seen directly), and shaded by both forms: the spectral
shade gives the reference XYZ; the latent shade of the encoded spectra,
decoded once, gives the codec's XYZ.  So every product of the chain runs in
the shading kernels, three bounces in one launch per form.

The CIE94 report per bounce (Sec. 4.5 compares the chains by CIE94) is a
host-side measurement, in CIELAB against an equal-energy white at the
luminance of the chain's light.
"""

from __future__ import annotations

import numpy as np
import torch

from . import colour, ops


def chain_paths(n_chains: int, bounces: int, device="cuda") -> ops.Paths:
    """Device records of the chains (see synth.chain_records for the layout)."""
    import synth
    hdr, pf, vtx = synth.chain_records(n_chains, bounces)
    return ops.Paths.from_numpy(hdr, pf, vtx, 1, device)


def chain_xyz(E, D, T, refl, lights, k: int, n: int, bounces: int = 3, paths=None):
    """XYZ of the chains in both forms.

    E (k x n), D (n x k), T (3 x n) float32; refl is (C * bounces, >= n)
    with chain c's reflectances in rows c * bounces + v, rows padded to a
    multiple of 4 floats; lights (C, >= n) likewise.  Returns torch tensors
    xyz_light (C, 3), xyz_spectral (bounces, C, 3), xyz_latent (bounces, C, 3).
    """
    C = lights.shape[0]
    if refl.shape[0] != C * bounces:
        raise ValueError(f"refl needs {C * bounces} rows (C x bounces), has {refl.shape[0]}")
    paths = paths or chain_paths(C, bounces, refl.device)
    xs = ops.shade_spectral(paths, refl, lights, T, n)
    xl = ops.shade_latent_xyz(paths, ops.encode(E, refl, n), ops.encode(E, lights, n),
                              ops.decode_matrix(D, T, k), k)
    return xs[:C], xs[C:].view(bounces, C, 3), xl[C:].view(bounces, C, 3)


def cie94_report(xyz_light, xyz_spectral, xyz_latent) -> list[dict]:
    """Per bounce: mean, p95 and max CIE94 of the latent chain against the
    spectral one.  Lab white: equal-energy, Y_n = Y of the chain's light;
    chains whose light has Y <= 0 are left out."""
    xl0 = np.asarray(torch.as_tensor(xyz_light).cpu(), dtype=np.float64)
    xs = np.asarray(torch.as_tensor(xyz_spectral).cpu(), dtype=np.float64)
    xl = np.asarray(torch.as_tensor(xyz_latent).cpu(), dtype=np.float64)
    keep = xl0[:, 1] > 0
    white = np.repeat(xl0[keep, 1:2], 3, axis=1)
    out = []
    for b in range(xs.shape[0]):
        d = colour.cie94(colour.xyz_to_lab(xs[b, keep], white), colour.xyz_to_lab(xl[b, keep], white))
        out.append(dict(bounce=b + 1, mean=float(d.mean()), p95=float(np.percentile(d, 95)),
                        max=float(d.max()), chains=int(d.size)))
    return out
