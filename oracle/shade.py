"""Oracle of encode, spectral shading, latent shading and decode (FP64).

Every array argument is converted to float64 before use.  Codes here are
plain k-vectors (channel c in column c); the blockwise product of Eq. 6
splits such a vector into B = k/3 triplets and multiplies them triplet by
triplet, which is the element-wise product of the whole vector.
"""

from __future__ import annotations

import numpy as np

from .records import unpack


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def encode(E, S):
    """Codes of the rows of S: z = W_enc s for each spectrum s (Eq. 4, left).

    E is k x n (W_enc), S is m x n; returns m x k.
    """
    return _f64(S) @ _f64(E).T


def decode(D, T, Z):
    """Decoded spectra s_hat = W_dec z (Eq. 4, right) and their XYZ = T_cmf s_hat.

    D is n x k (W_dec), T is 3 x n (T_cmf of the colour loss in Sec. 4.3),
    Z is m x k.  Returns (spectra m x n, xyz m x 3).
    """
    s_hat = _f64(Z) @ _f64(D).T
    return s_hat, s_hat @ _f64(T).T


def blockwise_product(za, zb):
    """Blockwise Hadamard product of Eq. 6: split both k-vectors into B = k/3
    triplets, multiply matching triplets element by element, concatenate."""
    za, zb = _f64(za), _f64(zb)
    k = za.shape[-1]
    if k % 3:
        raise ValueError("the blockwise product needs k = 3B")
    blocks = [za[..., 3 * i:3 * i + 3] * zb[..., 3 * i:3 * i + 3] for i in range(k // 3)]
    return np.concatenate(blocks, axis=-1)


def path_throughput(hdr, pix_first, vtx, spp, table, lights, product):
    """Per-path value: the light's vector times, for each vertex in path
    order, the vertex weight times the vertex's table row, combined with
    `product` (the element-wise product in spectral space, the blockwise one
    in code space).  This is the scale-and-multiply chain of Sec. 3 applied
    along a light path.  Returns (P, width) float64."""
    length, light, first, texel, weight = unpack(hdr, pix_first, vtx, spp)
    table, lights = _f64(table), _f64(lights)
    acc = lights[light].copy()
    for v in range(int(length.max()) if length.size else 0):
        live = np.flatnonzero(length > v)
        j = first[live] + v
        acc[live] = product(acc[live], weight[j][:, None] * table[texel[j]])
    return acc


def pixel_mean(per_path, spp):
    """Monte Carlo pixel estimate: mean over each pixel's spp samples."""
    p, w = per_path.shape
    return per_path.reshape(p // spp, spp, w).sum(axis=1) / spp


def shade_spectral(hdr, pix_first, vtx, spp, refl, illum, T):
    """Spectral form: XYZ_q = (1/spp) sum_{p in q} T_cmf (l_p * prod_v w_v r_v).

    refl is n_tex x n (reflectance rows), illum is n_illum x n, T is 3 x n.
    The spectral product is element-wise (Sec. 3); XYZ integration by the
    colour-matching matrix (Sec. 4.3).  Returns n_pixels x 3.
    """
    spec = path_throughput(hdr, pix_first, vtx, spp, refl, illum, np.multiply)
    return pixel_mean(spec @ _f64(T).T, spp)


def shade_latent(hdr, pix_first, vtx, spp, codes, light_codes):
    """Latent form: z_q = (1/spp) sum_{p in q} E(l_p) (.)_B prod_v w_v z_v.

    codes is n_tex x k (the encoded texels), light_codes is n_illum x k; the
    product is the blockwise Hadamard product of Eq. 6, so each 3-channel
    block is one RGB-style pass (Sec. 6.1).  Returns the n_pixels x k latent
    image (the re-assembled passes)."""
    z = path_throughput(hdr, pix_first, vtx, spp, codes, light_codes, blockwise_product)
    return pixel_mean(z, spp)


def render_latent_xyz(hdr, pix_first, vtx, spp, refl, illum, E, D, T):
    """End to end latent pipeline in FP64: encode the assets once, shade in
    code space, decode the latent image once (Fig. 2b).  Returns
    (latent image n_pixels x k, xyz n_pixels x 3)."""
    z = shade_latent(hdr, pix_first, vtx, spp, encode(E, refl), encode(E, illum))
    return z, decode(D, T, z)[1]
