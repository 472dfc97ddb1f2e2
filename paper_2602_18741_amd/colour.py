"""Colour-difference reports: XYZ -> CIELAB, CIEDE2000 and CIE94 (numpy, host).

These measure the method's approximation error (latent against spectral
images); they are reports, not part of the shading path.
"""

from __future__ import annotations

import numpy as np

_EPS = (6.0 / 29.0) ** 3


def xyz_to_lab(xyz, white):
    """CIE 1976 L*a*b* of XYZ rows relative to the white (Xn, Yn, Zn)."""
    xyz = np.asarray(xyz, dtype=np.float64) / np.asarray(white, dtype=np.float64)
    f = np.where(xyz > _EPS, np.cbrt(np.maximum(xyz, _EPS)), xyz / (3 * (6.0 / 29.0) ** 2) + 4.0 / 29.0)
    L = 116.0 * f[..., 1] - 16.0
    a = 500.0 * (f[..., 0] - f[..., 1])
    b = 200.0 * (f[..., 1] - f[..., 2])
    return np.stack([L, a, b], axis=-1)


def ciede2000(lab1, lab2, kL=1.0, kC=1.0, kH=1.0):
    """CIEDE2000 colour difference (Sharma, Wu and Dalal, Color Res. Appl.
    30(1), 2005), elementwise over the leading axes."""
    lab1 = np.asarray(lab1, dtype=np.float64)
    lab2 = np.asarray(lab2, dtype=np.float64)
    L1, a1, b1 = lab1[..., 0], lab1[..., 1], lab1[..., 2]
    L2, a2, b2 = lab2[..., 0], lab2[..., 1], lab2[..., 2]
    c_bar = 0.5 * (np.hypot(a1, b1) + np.hypot(a2, b2))
    c7 = c_bar ** 7
    g = 0.5 * (1.0 - np.sqrt(c7 / (c7 + 25.0 ** 7)))
    a1p, a2p = (1.0 + g) * a1, (1.0 + g) * a2
    c1p, c2p = np.hypot(a1p, b1), np.hypot(a2p, b2)
    h1p = np.where((a1p == 0) & (b1 == 0), 0.0, np.degrees(np.arctan2(b1, a1p)) % 360.0)
    h2p = np.where((a2p == 0) & (b2 == 0), 0.0, np.degrees(np.arctan2(b2, a2p)) % 360.0)
    dLp = L2 - L1
    dCp = c2p - c1p
    dh = h2p - h1p
    dh = np.where(dh > 180.0, dh - 360.0, np.where(dh < -180.0, dh + 360.0, dh))
    prod = c1p * c2p
    dh = np.where(prod == 0, 0.0, dh)
    dHp = 2.0 * np.sqrt(prod) * np.sin(np.radians(dh) / 2.0)
    Lbp = 0.5 * (L1 + L2)
    Cbp = 0.5 * (c1p + c2p)
    hsum = h1p + h2p
    hbp = np.where(prod == 0, hsum,
                   np.where(np.abs(h1p - h2p) <= 180.0, hsum / 2.0,
                            np.where(hsum < 360.0, (hsum + 360.0) / 2.0, (hsum - 360.0) / 2.0)))
    T = (1.0 - 0.17 * np.cos(np.radians(hbp - 30.0)) + 0.24 * np.cos(np.radians(2.0 * hbp))
         + 0.32 * np.cos(np.radians(3.0 * hbp + 6.0)) - 0.20 * np.cos(np.radians(4.0 * hbp - 63.0)))
    dtheta = 30.0 * np.exp(-(((hbp - 275.0) / 25.0) ** 2))
    cb7 = Cbp ** 7
    Rc = 2.0 * np.sqrt(cb7 / (cb7 + 25.0 ** 7))
    Sl = 1.0 + 0.015 * (Lbp - 50.0) ** 2 / np.sqrt(20.0 + (Lbp - 50.0) ** 2)
    Sc = 1.0 + 0.045 * Cbp
    Sh = 1.0 + 0.015 * Cbp * T
    Rt = -np.sin(np.radians(2.0 * dtheta)) * Rc
    tl, tc, th = dLp / (kL * Sl), dCp / (kC * Sc), dHp / (kH * Sh)
    return np.sqrt(np.maximum(tl * tl + tc * tc + th * th + Rt * tc * th, 0.0))


def cie94(lab_ref, lab, kL=1.0, kC=1.0, kH=1.0):
    """CIE94 colour difference (graphic-arts weights) of lab against lab_ref."""
    lab_ref = np.asarray(lab_ref, dtype=np.float64)
    lab = np.asarray(lab, dtype=np.float64)
    dL = lab_ref[..., 0] - lab[..., 0]
    c1 = np.hypot(lab_ref[..., 1], lab_ref[..., 2])
    c2 = np.hypot(lab[..., 1], lab[..., 2])
    dC = c1 - c2
    da = lab_ref[..., 1] - lab[..., 1]
    db = lab_ref[..., 2] - lab[..., 2]
    dH2 = np.maximum(da * da + db * db - dC * dC, 0.0)
    sC = 1.0 + 0.045 * c1
    sH = 1.0 + 0.015 * c1
    return np.sqrt((dL / kL) ** 2 + (dC / (kC * sC)) ** 2 + dH2 / (kH * sH) ** 2)


def frame_difference(xyz_ref, xyz, metric=ciede2000):
    """Colour difference of an image against a reference image.

    Both are converted to Lab with an equal-energy white scaled to the
    reference's largest Y (shared by both); pixels with reference Y <= 0 are
    ignored.  Returns dict(mean, p95, max, pixels)."""
    xyz_ref = np.asarray(xyz_ref, dtype=np.float64).reshape(-1, 3)
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    keep = xyz_ref[:, 1] > 0
    yn = xyz_ref[keep, 1].max() if keep.any() else 1.0
    white = np.array([yn, yn, yn])
    d = metric(xyz_to_lab(xyz_ref[keep], white), xyz_to_lab(xyz[keep], white))
    if d.size == 0:
        return dict(mean=0.0, p95=0.0, max=0.0, pixels=0)
    return dict(mean=float(d.mean()), p95=float(np.percentile(d, 95)), max=float(d.max()),
                pixels=int(d.size))
