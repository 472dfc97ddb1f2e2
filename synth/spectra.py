"""Spectra, colour-matching table and codec matrices (input data only)."""

from __future__ import annotations

import numpy as np

# Second radiation constant c2 = h c / k_B in metre-kelvin (CODATA).
C2_M_K = 1.438777e-2


def wavelengths(n: int) -> np.ndarray:
    """Uniform wavelength grid in nm for the two sample counts the workloads use.

    n = 31: 400..700 nm in 10 nm steps (the paper zeroes its spectra outside
    400-700 nm, Sec. 4.4, which leaves 31 samples at 10 nm).
    n = 81: 380..780 nm in 5 nm steps (the visible range named in Sec. 1).
    Any other n spreads n samples uniformly over 400..700 nm.
    """
    if n == 31:
        return np.arange(400.0, 701.0, 10.0)
    if n == 81:
        return np.arange(380.0, 781.0, 5.0)
    if n == 1:
        return np.array([550.0])
    return np.linspace(400.0, 700.0, n)


def _lobe(lam: np.ndarray, mu: float, s_lo: float, s_hi: float) -> np.ndarray:
    sigma = np.where(lam < mu, s_lo, s_hi)
    t = (lam - mu) / sigma
    return np.exp(-0.5 * t * t)


def cmf_fit_cie1931(lam: np.ndarray) -> np.ndarray:
    """CIE 1931 2-degree colour-matching functions, analytic multi-lobe fit.

    Piecewise-Gaussian lobes of Wyman, Sloan and Shirley, "Simple Analytic
    Approximations to the CIE XYZ Color Matching Functions", JCGT 2(2), 2013.
    Returns a (3, n) float64 array [xbar, ybar, zbar].
    """
    lam = np.asarray(lam, dtype=np.float64)
    x = (1.056 * _lobe(lam, 599.8, 37.9, 31.0)
         + 0.362 * _lobe(lam, 442.0, 16.0, 26.7)
         - 0.065 * _lobe(lam, 501.1, 20.4, 26.2))
    y = 0.821 * _lobe(lam, 568.8, 46.9, 40.5) + 0.286 * _lobe(lam, 530.9, 16.3, 31.1)
    z = 1.217 * _lobe(lam, 437.0, 11.8, 36.0) + 0.681 * _lobe(lam, 459.0, 26.0, 13.8)
    return np.stack([x, y, z])


def cmf_matrix(n: int) -> np.ndarray:
    """The colour-matching matrix T (3 x n, float32) used as an input table.

    T[c, i] = cmf_c(lambda_i) / sum_j ybar(lambda_j): the rectangle rule with
    the wavelength step cancelled, so a unit equal-energy spectrum has Y = 1.
    The paper only names this matrix (T_cmf in R^{3 x n}, Sec. 4.3 colour
    loss); the quadrature and normalisation are a choice of this input.
    """
    cmf = cmf_fit_cie1931(wavelengths(n))
    return (cmf / cmf[1].sum()).astype(np.float32)


def planck(lam_nm: np.ndarray, temp_k: float) -> np.ndarray:
    """Planck's law up to a constant, normalised to peak 1 over the grid samples."""
    lam = np.asarray(lam_nm, dtype=np.float64) * 1e-9
    b = lam ** -5 / np.expm1(C2_M_K / (lam * temp_k))
    return b / b.max()


def gaussian_mixture(rng: np.random.Generator, lam: np.ndarray, count: int,
                     sigma_lo: float, sigma_hi: float, chunk: int = 65536) -> np.ndarray:
    """`count` spectra, each a sum of 1-3 Gaussian lobes.

    Lobe count uniform in {1, 2, 3}; centre U[400, 700] nm, width sigma
    U[sigma_lo, sigma_hi] nm, amplitude U[0, 1].  The draws are taken in the
    order: lobe counts (count,), centres (count, 3), widths (count, 3),
    amplitudes (count, 3); lobes beyond a spectrum's count get amplitude 0.
    Returns (count, n) float64.
    """
    lam = np.asarray(lam, dtype=np.float64)
    n_lobes = rng.integers(1, 4, size=count)
    mu = rng.uniform(400.0, 700.0, size=(count, 3))
    sig = rng.uniform(sigma_lo, sigma_hi, size=(count, 3))
    amp = rng.uniform(0.0, 1.0, size=(count, 3))
    amp = amp * (np.arange(3)[None, :] < n_lobes[:, None])
    out = np.empty((count, lam.size))
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        t = (lam[None, None, :] - mu[c0:c1, :, None]) / sig[c0:c1, :, None]
        out[c0:c1] = np.einsum("cl,cln->cn", amp[c0:c1], np.exp(-0.5 * t * t))
    return out


def reflectances(rng: np.random.Generator, n: int, count: int) -> np.ndarray:
    """Broad reflectance spectra: 1-3 lobes, sigma U[20, 80] nm, clipped to [0, 1]."""
    r = gaussian_mixture(rng, wavelengths(n), count, 20.0, 80.0)
    return np.clip(r, 0.0, 1.0).astype(np.float32)


def narrowband(rng: np.random.Generator, n: int, count: int,
               sigma_lo: float = 5.0, sigma_hi: float = 15.0) -> np.ndarray:
    """Narrow-band light spectra (1-3 lobes), each normalised to unit peak."""
    s = gaussian_mixture(rng, wavelengths(n), count, sigma_lo, sigma_hi)
    peak = s.max(axis=1, keepdims=True)
    peak[peak == 0.0] = 1.0
    return (s / peak).astype(np.float32)


def planck_table(lam_nm: np.ndarray, temps: np.ndarray) -> np.ndarray:
    """Rows of `planck` for each temperature in `temps` (vectorised)."""
    lam = np.asarray(lam_nm, dtype=np.float64)[None, :] * 1e-9
    b = lam ** -5 / np.expm1(C2_M_K / (lam * np.asarray(temps, dtype=np.float64)[:, None]))
    return b / b.max(axis=1, keepdims=True)


def illuminant_table(rng: np.random.Generator, n: int, n_planck: int, n_narrow: int,
                     sigma_lo: float = 5.0, sigma_hi: float = 15.0) -> np.ndarray:
    """Light table: ids [0, n_planck) Planckian at T ~ U[2500, 9000] K, then
    n_narrow narrow-band mixtures.  All unit-peak on the grid (Sec. 4.4 lights
    are normalised to unit peak).  Returns (n_planck + n_narrow, n) float32."""
    lam = wavelengths(n)
    temps = rng.uniform(2500.0, 9000.0, size=n_planck)
    pl = planck_table(lam, temps) if n_planck else np.zeros((0, n))
    nb = narrowband(rng, n, n_narrow, sigma_lo, sigma_hi)
    return np.concatenate([pl.astype(np.float32), nb], axis=0)


def codec_uniform(rng: np.random.Generator, k: int, n: int):
    """Random non-negative codec: E (k x n) and D (n x k) with entries U[0, 1]."""
    e = rng.uniform(0.0, 1.0, size=(k, n)).astype(np.float32)
    d = rng.uniform(0.0, 1.0, size=(n, k)).astype(np.float32)
    return e, d


def codec_init(rng: np.random.Generator, k: int, n: int, std: float = 0.1):
    """Unconstrained codec parameters W~_E (k x n), W~_D (n x k) ~ N(0, std^2)."""
    we = rng.normal(0.0, std, size=(k, n)).astype(np.float32)
    wd = rng.normal(0.0, std, size=(n, k)).astype(np.float32)
    return we, wd


# XYZ -> linear sRGB primaries (IEC 61966-2-1, the published 4-decimal matrix).
XYZ_TO_LINEAR_SRGB = np.array([[3.2406, -1.5372, -0.4986],
                               [-0.9689, 1.8758, 0.0415],
                               [0.0557, -0.2040, 1.0570]])
