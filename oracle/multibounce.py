"""Oracle of the multi-bounce evaluation chain (Eq. 10, Sec. 4.5), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A chain starts from a light spectrum L and meets reflectances R_1, R_2, ...
in turn; after b bounces the spectral radiance is S_b = R_b * S_{b-1} with
S_0 = L (element-wise products, Eq. 10).  The latent form runs the same
recurrence on codes: z_0 = E L, z_b = E R_b (.)_B z_{b-1} (blockwise
product, Eq. 6), decoded once at the end, s_hat_b = D z_b (Eq. 4).  Both are
projected to XYZ with the colour-matching matrix T.
"""

from __future__ import annotations

import numpy as np

from .shade import blockwise_product


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def chain_xyz(R, L, E, D, T):
    """R: (C, bounces, n) reflectances in the order met; L: (C, n) lights;
    E (k x n), D (n x k), T (3 x n).  A k that is not a multiple of 3 is
    padded with zero channels (zero rows of E, zero columns of D), which
    carry 0 through every product and the decode.

    Returns (xyz_light (C, 3) = T L, xyz_spectral (bounces, C, 3),
    xyz_latent (bounces, C, 3))."""
    R, L, E, D, T = _f64(R), _f64(L), _f64(E), _f64(D), _f64(T)
    k = E.shape[0]
    pad = (-k) % 3
    if pad:
        E = np.vstack([E, np.zeros((pad, E.shape[1]))])
        D = np.hstack([D, np.zeros((D.shape[0], pad))])
    bounces = R.shape[1]
    S = L.copy()
    z = L @ E.T
    xs, xl = [], []
    for b in range(bounces):
        S = R[:, b] * S
        z = blockwise_product(R[:, b] @ E.T, z)
        xs.append(S @ T.T)
        xl.append((z @ D.T) @ T.T)
    return L @ T.T, np.stack(xs), np.stack(xl)
