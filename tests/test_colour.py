"""Closed-form cases of the colour-difference reports (no GPU)."""

import numpy as np
import pytest

from paper_2602_18741_amd import colour


def test_white_and_black_lab():
    white = np.array([0.9, 1.0, 1.1])
    assert np.allclose(colour.xyz_to_lab(white, white), [100.0, 0.0, 0.0], atol=1e-12)
    assert np.allclose(colour.xyz_to_lab(np.zeros(3), white), [0.0, 0.0, 0.0], atol=1e-12)
    # the linear segment joins the cube root at (6/29)^3
    t = (6 / 29) ** 3
    lab = colour.xyz_to_lab(np.array([t, t, t]), np.ones(3))
    assert lab[0] == pytest.approx(116 * 6 / 29 - 16, rel=1e-12)


def test_ciede2000_identity_and_symmetry():
    rng = np.random.default_rng(0)
    a = np.stack([rng.uniform(0, 100, 500), rng.uniform(-80, 80, 500), rng.uniform(-80, 80, 500)], 1)
    b = a + rng.normal(0, 5, a.shape)
    assert np.all(colour.ciede2000(a, a) == 0)
    assert np.allclose(colour.ciede2000(a, b), colour.ciede2000(b, a), rtol=1e-12, atol=1e-12)
    assert np.all(colour.ciede2000(a, b) > 0)


def test_ciede2000_neutral_lightness_closed_form():
    """Neutral colours (a* = b* = 0) differing only in L*: every chroma and
    hue term vanishes and the difference is |dL| / S_L with
    S_L = 1 + 0.015 (Lbar - 50)^2 / sqrt(20 + (Lbar - 50)^2)."""
    for L1, L2 in [(40.0, 60.0), (10.0, 15.0), (70.0, 95.0)]:
        lb = 0.5 * (L1 + L2)
        sl = 1 + 0.015 * (lb - 50) ** 2 / np.sqrt(20 + (lb - 50) ** 2)
        d = colour.ciede2000(np.array([L1, 0, 0]), np.array([L2, 0, 0]))
        assert d == pytest.approx(abs(L2 - L1) / sl, rel=1e-12)
    assert colour.ciede2000(np.array([45.0, 0, 0]), np.array([55.0, 0, 0])) == pytest.approx(10.0)


def test_ciede2000_chroma_on_the_axes_closed_forms():
    """Equal lightness, both colours on the positive a* axis (b* = 0): both
    hue angles are 0, so the hue difference and the rotation term vanish and
    the difference is |dC'| / S_C with a' = (1 + G) a,
    G = (1 - sqrt(Cbar^7 / (Cbar^7 + 25^7))) / 2 (Cbar the mean of the two
    chromas before the adjustment) and S_C = 1 + 0.045 Cbar'.  On the b*
    axis (a* = 0) the adjustment, which scales a* only, has no effect:
    |db| / (1 + 0.045 (b1 + b2) / 2)."""
    for a1, a2 in [(10.0, 14.0), (30.0, 42.0), (2.0, 3.0)]:
        cbar = 0.5 * (a1 + a2)
        G = 0.5 * (1 - np.sqrt(cbar ** 7 / (cbar ** 7 + 25.0 ** 7)))
        c1, c2 = (1 + G) * a1, (1 + G) * a2
        want = abs(c2 - c1) / (1 + 0.045 * 0.5 * (c1 + c2))
        got = colour.ciede2000(np.array([50.0, a1, 0.0]), np.array([50.0, a2, 0.0]))
        assert got == pytest.approx(want, rel=1e-12)
    for b1, b2 in [(10.0, 14.0), (30.0, 42.0)]:
        want = abs(b2 - b1) / (1 + 0.045 * 0.5 * (b1 + b2))
        got = colour.ciede2000(np.array([60.0, 0.0, b1]), np.array([60.0, 0.0, b2]))
        assert got == pytest.approx(want, rel=1e-12)


def test_cie94_lightness_only_and_zero():
    a = np.array([50.0, 20.0, -10.0])
    assert colour.cie94(a, a) == 0.0
    assert colour.cie94(a, a + [3.0, 0, 0]) == pytest.approx(3.0, rel=1e-12)


def test_frame_difference_ignores_black_reference_pixels():
    ref = np.array([[0.2, 0.3, 0.1], [0.0, 0.0, 0.0], [0.5, 0.4, 0.9]])
    d = colour.frame_difference(ref, ref)
    assert d["pixels"] == 2 and d["mean"] == 0.0


def test_cie94_chroma_and_hue_closed_forms():
    """At equal lightness: a pure chroma change (same hue angle) gives
    |dC| / (1 + 0.045 C_ref); a pure hue rotation (same chroma) gives
    |da, db| / (1 + 0.015 C_ref), since then dH^2 = da^2 + db^2."""
    c1, c2, h = 30.0, 36.0, np.radians(40.0)
    ref = np.array([50.0, c1 * np.cos(h), c1 * np.sin(h)])
    chroma = np.array([50.0, c2 * np.cos(h), c2 * np.sin(h)])
    assert colour.cie94(ref, chroma) == pytest.approx(abs(c2 - c1) / (1 + 0.045 * c1), rel=1e-12)
    g = np.radians(55.0)
    hue = np.array([50.0, c1 * np.cos(g), c1 * np.sin(g)])
    dab = np.hypot(*(hue[1:] - ref[1:]))
    assert colour.cie94(ref, hue) == pytest.approx(dab / (1 + 0.015 * c1), rel=1e-12)
