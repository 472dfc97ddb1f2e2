"""Pins of the multi-bounce chain oracle (Eq. 10) (no GPU)."""

import numpy as np
import pytest

import synth
from oracle import multibounce as mb
from oracle import shade


def _chains(n, C, bounces, seed):
    rng = np.random.default_rng(seed)
    R = synth.reflectances(rng, n, C * bounces).reshape(C, bounces, n)
    L = synth.illuminant_table(rng, n, C // 2, C - C // 2)
    return R.astype(np.float64), L.astype(np.float64)


def test_identity_codec_reproduces_the_spectral_chain():
    """E = D = I (k = n = 31, padded to 33 channels): every latent product is
    the spectral one, so the two XYZ chains coincide."""
    n = 31
    R, L = _chains(n, 40, 3, 0)
    T = synth.cmf_matrix(n)
    xl0, xs, xl = mb.chain_xyz(R, L, np.eye(n), np.eye(n), T)
    assert np.allclose(xl, xs, rtol=1e-14, atol=0)
    assert np.allclose(xl0, L @ T.astype(np.float64).T, rtol=1e-15, atol=0)


def test_constant_spectra_closed_form():
    """R_b = c_b 1 and L = l 1: S_b = l c_1 ... c_b 1, so
    XYZ_b = l prod(c) T 1; in code space z_b = l prod(c) (E 1)^(b+1)
    (element-wise power), so XYZ_b = l prod(c) T D (E 1)^(b+1)."""
    n, k, C = 31, 6, 5
    rng = np.random.default_rng(1)
    c = rng.uniform(0.2, 1.0, (C, 3))
    lv = rng.uniform(0.5, 2.0, C)
    R = c[:, :, None] * np.ones((C, 3, n))
    L = lv[:, None] * np.ones((C, n))
    E, D = rng.uniform(size=(k, n)), rng.uniform(size=(n, k))
    T = synth.cmf_matrix(n).astype(np.float64)
    _, xs, xl = mb.chain_xyz(R, L, E, D, T)
    e1 = E @ np.ones(n)
    for b in range(3):
        scale = lv * c[:, :b + 1].prod(axis=1)
        assert np.allclose(xs[b], scale[:, None] * (T @ np.ones(n))[None, :], rtol=1e-14, atol=0)
        assert np.allclose(xl[b], scale[:, None] * (T @ D @ e1 ** (b + 2))[None, :], rtol=1e-13, atol=0)


def test_box_spectra_closed_form():
    """Indicator spectra: the chain after b bounces is the indicator of the
    intersection of the light's and the first b reflectances' intervals, so
    XYZ_b = sum of T's columns over that intersection."""
    n, C = 31, 30
    rng = np.random.default_rng(2)
    lo = rng.integers(0, 20, (C, 4))
    hi = lo + rng.integers(3, 12, (C, 4))
    idx = np.arange(n)
    box = ((idx[None, None, :] >= lo[..., None]) & (idx[None, None, :] < hi[..., None])).astype(float)
    L, R = box[:, 0], box[:, 1:]
    T = synth.cmf_matrix(n).astype(np.float64)
    _, xs, _ = mb.chain_xyz(R, L, np.eye(n), np.eye(n), T)
    for b in range(3):
        inter = box[:, :b + 2].prod(axis=1)
        assert np.allclose(xs[b], inter @ T.T, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,k", [(31, 6), (81, 9)])
def test_chain_equals_the_path_renderer_on_chain_records(n, k):
    """The recurrence against the record-driven renderers of the oracle,
    fed the chain records: pixel b * C + c holds chain c after b bounces."""
    C, bounces = 24, 3
    R, L = _chains(n, C, bounces, 3)
    rng = np.random.default_rng(4)
    E, D = rng.uniform(size=(k, n)), rng.uniform(size=(n, k))
    T = synth.cmf_matrix(n)
    hdr, pf, vtx = synth.chain_records(C, bounces)
    refl = R.reshape(C * bounces, n)
    spec = shade.shade_spectral(hdr, pf, vtx, 1, refl, L, T)
    _, lat = shade.render_latent_xyz(hdr, pf, vtx, 1, refl, L, E, D, T)
    x0, xs, xl = mb.chain_xyz(R, L, E, D, T)
    assert np.allclose(spec[:C], x0, rtol=1e-14, atol=0)
    assert np.allclose(spec[C:].reshape(bounces, C, 3), xs, rtol=1e-13, atol=0)
    assert np.allclose(lat[C:].reshape(bounces, C, 3), xl, rtol=1e-13, atol=0)
