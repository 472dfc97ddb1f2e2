"""Pins of the oracle's encode / shade / decode against closed forms,
invariants and exact rational brute force (no GPU)."""

from fractions import Fraction
import itertools

import numpy as np
import pytest

import synth
from oracle import records, shade


def _records(paths, spp):
    """Pack per-path (light, [(texel, weight), ...]) into the record format."""
    hdr, vtx, pix_first = [], [], []
    for q in range(len(paths) // spp):
        pix_first.append(len(vtx))
        for light, verts in paths[q * spp:(q + 1) * spp]:
            hdr.append(light | (len(verts) << 24))
            for t, w in verts:
                vtx.append((t, np.float32(w).view(np.uint32)))
    return (np.array(hdr, dtype=np.uint32), np.array(pix_first, dtype=np.uint32),
            np.array(vtx, dtype=np.uint32).reshape(-1, 2))


def _random_scene(rng, n_px, spp, lmax, n_tex, n_illum, lmin=1):
    paths = []
    for _ in range(n_px * spp):
        L = int(rng.integers(lmin, lmax + 1))
        verts = [(int(rng.integers(n_tex)), float(np.float32(rng.uniform()))) for _ in range(L)]
        paths.append((int(rng.integers(n_illum)), verts))
    return paths


# ---------------------------------------------------------------- encode / decode

def test_encode_basis_vectors_give_columns():
    """z = W_enc e_i is column i of W_enc (Eq. 4); a transposed operand fails."""
    rng = np.random.default_rng(0)
    E = rng.uniform(size=(6, 31)).astype(np.float32)
    Z = shade.encode(E, np.eye(31, dtype=np.float32))
    assert Z.shape == (31, 6)
    for i in range(31):
        assert np.array_equal(Z[i], E[:, i].astype(np.float64))


def test_encode_is_linear():
    """Scaling and addition map exactly to codes (Sec. 4.1), to rounding."""
    rng = np.random.default_rng(1)
    E = rng.uniform(size=(9, 31))
    s, t = rng.uniform(size=(2, 50, 31))
    a, b = 0.37, 2.5
    lhs = shade.encode(E, a * s + b * t)
    rhs = a * shade.encode(E, s) + b * shade.encode(E, t)
    assert np.allclose(lhs, rhs, rtol=1e-13, atol=0)


def test_encode_identity_is_exact():
    S = np.random.default_rng(2).uniform(size=(20, 12)).astype(np.float32)
    assert np.array_equal(shade.encode(np.eye(12), S), S.astype(np.float64))


def test_decode_box_columns():
    """Decoder column c set to the indicator of an index set: decoding e_c
    gives that indicator and XYZ = sum of T's columns over the set."""
    rng = np.random.default_rng(3)
    n, k = 31, 6
    T = rng.integers(0, 7, size=(3, n)).astype(np.float64)
    sets = [sorted(rng.choice(n, size=int(rng.integers(1, n)), replace=False)) for _ in range(k)]
    D = np.zeros((n, k))
    for c, idx in enumerate(sets):
        D[idx, c] = 1.0
    s_hat, xyz = shade.decode(D, T, np.eye(k))
    for c, idx in enumerate(sets):
        want = np.zeros(n)
        want[idx] = 1.0
        assert np.array_equal(s_hat[c], want)
        assert np.array_equal(xyz[c], sum(T[:, i] for i in idx))


def test_decode_commutes_with_pixel_mean():
    """decode(mean z) = mean decode(z), by linearity (Sec. 4.1)."""
    rng = np.random.default_rng(4)
    D, T = rng.uniform(size=(31, 6)), rng.uniform(size=(3, 31))
    z = rng.uniform(size=(16, 6))
    a = shade.decode(D, T, z.mean(axis=0, keepdims=True))[1]
    b = shade.decode(D, T, z)[1].mean(axis=0, keepdims=True)
    assert np.allclose(a, b, rtol=1e-14)


# ---------------------------------------------------------------- spectral shading

def test_spectral_box_spectra_closed_form():
    """Indicator spectra: the path spectrum is prod(w) on the intersection of
    the intervals, so XYZ = prod(w) * sum of T's columns over it."""
    rng = np.random.default_rng(5)
    n, n_tex, n_illum = 31, 12, 4
    T = rng.uniform(size=(3, n)).astype(np.float32)

    def box():
        a = int(rng.integers(0, n - 1))
        b = int(rng.integers(a + 1, n + 1))
        row = np.zeros(n, dtype=np.float32)
        row[a:b] = 1.0
        return (a, b), row

    tex = [box() for _ in range(n_tex)]
    lig = [box() for _ in range(n_illum)]
    refl = np.stack([r for _, r in tex])
    illum = np.stack([r for _, r in lig])
    paths = _random_scene(rng, 64, 1, 4, n_tex, n_illum)
    hdr, pf, vtx = _records(paths, 1)
    got = shade.shade_spectral(hdr, pf, vtx, 1, refl, illum, T)
    for q, (light, verts) in enumerate(paths):
        lo, hi = lig[light][0]
        wprod = 1.0
        for t, w in verts:
            lo, hi = max(lo, tex[t][0][0]), min(hi, tex[t][0][1])
            wprod *= float(np.float32(w))
        want = wprod * T[:, lo:hi].astype(np.float64).sum(axis=1) if hi > lo else np.zeros(3)
        assert np.allclose(got[q], want, rtol=1e-13, atol=1e-300)


def test_spectral_constant_spectra():
    """Constant spectra: x = a * prod(w c) * T 1."""
    rng = np.random.default_rng(6)
    n = 31
    T = synth.cmf_matrix(n)
    cvals = rng.uniform(size=8).astype(np.float32)
    avals = rng.uniform(size=3).astype(np.float32)
    refl = np.repeat(cvals[:, None], n, axis=1)
    illum = np.repeat(avals[:, None], n, axis=1)
    paths = _random_scene(rng, 40, 1, 5, 8, 3)
    hdr, pf, vtx = _records(paths, 1)
    got = shade.shade_spectral(hdr, pf, vtx, 1, refl, illum, T)
    t1 = T.astype(np.float64).sum(axis=1)
    for q, (light, verts) in enumerate(paths):
        f = float(avals[light])
        for t, w in verts:
            f *= float(np.float32(w)) * float(cvals[t])
        assert np.allclose(got[q], f * t1, rtol=1e-13)


@pytest.mark.parametrize("spp", [1, 2, 4])
def test_spectral_exact_rational_brute_force(spp):
    """2x2 pixels, every light x material combination reachable, evaluated in
    exact rationals from the float32 inputs; the oracle agrees to 1e-14."""
    rng = np.random.default_rng(10 + spp)
    n, n_tex, n_illum = 5, 3, 2
    refl = rng.uniform(size=(n_tex, n)).astype(np.float32)
    illum = rng.uniform(size=(n_illum, n)).astype(np.float32)
    T = rng.uniform(size=(3, n)).astype(np.float32)
    combos = [(l, m) for l, m in itertools.product(range(n_illum), range(n_tex))]
    paths = []
    for p in range(4 * spp):
        l, m = combos[p % len(combos)]
        L = 1 + p % 3
        verts = [((m + v) % n_tex, float(np.float32(rng.uniform()))) for v in range(L)]
        paths.append((l, verts))
    hdr, pf, vtx = _records(paths, spp)
    got = shade.shade_spectral(hdr, pf, vtx, spp, refl, illum, T)
    F = Fraction
    for q in range(4):
        acc = [F(0)] * 3
        for light, verts in paths[q * spp:(q + 1) * spp]:
            s = [F(float(illum[light, i])) for i in range(n)]
            for t, w in verts:
                s = [s[i] * F(float(np.float32(w))) * F(float(refl[t, i])) for i in range(n)]
            for c in range(3):
                acc[c] += sum(F(float(T[c, i])) * s[i] for i in range(n))
        want = np.array([float(a / spp) for a in acc])
        assert np.allclose(got[q], want, rtol=1e-14, atol=0)


def test_spectral_pixel_is_mean_of_samples():
    """A pixel whose spp samples are copies of one path equals that path at
    spp = 1, and the sample order inside a pixel does not matter."""
    w = synth.workload(0)
    rng = np.random.default_rng(7)
    base = _random_scene(rng, 8, 1, 3, w["n_tex"], 8)
    hdr1, pf1, vtx1 = _records(base, 1)
    one = shade.shade_spectral(hdr1, pf1, vtx1, 1, w["refl"], w["illum"], w["T"])
    rep = [p for p in base for _ in range(4)]
    hdr4, pf4, vtx4 = _records(rep, 4)
    four = shade.shade_spectral(hdr4, pf4, vtx4, 4, w["refl"], w["illum"], w["T"])
    assert np.allclose(one, four, rtol=1e-15)
    mixed = _random_scene(rng, 4, 4, 3, w["n_tex"], 8)
    shuffled = [mixed[q * 4 + j] for q in range(4) for j in (2, 0, 3, 1)]
    a = shade.shade_spectral(*_records(mixed, 4), 4, w["refl"], w["illum"], w["T"])
    b = shade.shade_spectral(*_records(shuffled, 4), 4, w["refl"], w["illum"], w["T"])
    assert np.allclose(a, b, rtol=1e-14)


def test_zero_length_path_sees_the_light():
    w = synth.workload(0)
    paths = [(3, []), (5, [])]
    got = shade.shade_spectral(*_records(paths, 1), 1, w["refl"], w["illum"], w["T"])
    T = w["T"].astype(np.float64)
    assert np.allclose(got[0], T @ w["illum"][3], rtol=1e-14)
    assert np.allclose(got[1], T @ w["illum"][5], rtol=1e-14)


# ---------------------------------------------------------------- latent shading

def _identity_codec(n):
    k = 3 * ((n + 2) // 3)
    E = np.zeros((k, n))
    E[:n, :n] = np.eye(n)
    return E, E.T.copy()


def test_identity_codec_latent_equals_spectral():
    """k = n (padded to 3B with zero channels) and E = D = I: the latent
    pipeline reproduces the spectral one (the special case of Eqs. 4 and 6
    where the blockwise product is the spectral product)."""
    w = synth.workload(0, width=32, height=16, spp=4)
    spec = synth.PathSpec(n_pixels=512, spp=4, l_min=0, l_max=4, n_tex=64, n_illum=8, seed=99)
    hdr, pf, vtx = synth.gen_paths(spec)
    E, D = _identity_codec(31)
    ref = shade.shade_spectral(hdr, pf, vtx, 4, w["refl"], w["illum"], w["T"])
    _, got = shade.render_latent_xyz(hdr, pf, vtx, 4, w["refl"], w["illum"], E, D, w["T"])
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-300)


def test_single_vertex_reduces_to_decoded_code():
    """Light code = the multiplicative identity 1_k and L = 1: the latent
    pixel is w z_t, so XYZ = T D E (w r_t)."""
    w = synth.workload(0)
    rng = np.random.default_rng(8)
    E, D, T, refl = w["E"], w["D"], w["T"], w["refl"]
    paths = _random_scene(rng, 32, 1, 1, w["n_tex"], 1)
    hdr, pf, vtx = _records(paths, 1)
    codes = shade.encode(E, refl)
    z = shade.shade_latent(hdr, pf, vtx, 1, codes, np.ones((1, 6)))
    xyz = shade.decode(D, T, z)[1]
    for q, (_, [(t, wt)]) in enumerate(paths):
        s = float(np.float32(wt)) * refl[t].astype(np.float64)
        want = T.astype(np.float64) @ (D.astype(np.float64) @ (E.astype(np.float64) @ s))
        assert np.allclose(xyz[q], want, rtol=1e-13)


def test_blocks_are_independent_passes():
    """Eq. 6: each 3-channel block multiplies only within itself, so shading
    the two halves of a k = 6 code separately and concatenating the images
    equals shading the whole code (the B render passes of Sec. 6.1)."""
    w = synth.workload(0)
    spec = synth.PathSpec(n_pixels=300, spp=2, l_min=1, l_max=4, n_tex=64, n_illum=8, seed=5)
    hdr, pf, vtx = synth.gen_paths(spec)
    codes = shade.encode(w["E"], w["refl"])
    lc = shade.encode(w["E"], w["illum"])
    full = shade.shade_latent(hdr, pf, vtx, 2, codes, lc)
    halves = [shade.shade_latent(hdr, pf, vtx, 2, codes[:, b:b + 3], lc[:, b:b + 3]) for b in (0, 3)]
    assert np.array_equal(full, np.concatenate(halves, axis=1))


def test_latent_exact_rational_brute_force():
    rng = np.random.default_rng(20)
    k = 6
    codes = rng.uniform(size=(4, k)).astype(np.float32)
    lc = rng.uniform(size=(2, k)).astype(np.float32)
    paths = _random_scene(rng, 4, 2, 3, 4, 2, lmin=0)
    hdr, pf, vtx = _records(paths, 2)
    got = shade.shade_latent(hdr, pf, vtx, 2, codes, lc)
    F = Fraction
    for q in range(4):
        acc = [F(0)] * k
        for light, verts in paths[2 * q:2 * q + 2]:
            z = [F(float(lc[light, c])) for c in range(k)]
            for t, wt in verts:
                z = [z[c] * F(float(np.float32(wt))) * F(float(codes[t, c])) for c in range(k)]
            acc = [a + b for a, b in zip(acc, z)]
        assert np.allclose(got[q], [float(a / 2) for a in acc], rtol=1e-14, atol=0)


def test_non_negativity():
    """Non-negative spectra and codec give non-negative codes, spectra and XYZ
    (Sec. 4.1, 4.3); the fitted CMF table is non-negative on both grids."""
    w = synth.workload(0)
    spec = synth.PathSpec(n_pixels=256, spp=2, l_min=1, l_max=3, n_tex=64, n_illum=8, seed=3)
    hdr, pf, vtx = synth.gen_paths(spec)
    z, xyz = shade.render_latent_xyz(hdr, pf, vtx, 2, w["refl"], w["illum"], w["E"], w["D"], w["T"])
    assert (z >= 0).all() and (xyz >= 0).all()
    assert (shade.shade_spectral(hdr, pf, vtx, 2, w["refl"], w["illum"], w["T"]) >= 0).all()
    assert (synth.cmf_matrix(31) >= 0).all() and (synth.cmf_matrix(81) >= 0).all()


# ---------------------------------------------------------------- records

def test_record_check_counts_planted_errors():
    spec = synth.PathSpec(n_pixels=100, spp=4, l_min=1, l_max=4, n_tex=64, n_illum=8, seed=11)
    hdr, pf, vtx = synth.gen_paths(spec)
    assert records.check(hdr, pf, vtx, 4, 64, 8) == (0, 0, 0)
    hdr, pf, vtx = hdr.copy(), pf.copy(), vtx.copy()
    hdr[[3, 17]] = (hdr[[3, 17]] & 0xFF000000) | 8     # light id 8 of 8
    vtx[[0, 5, 6], 0] = 64                              # texel 64 of 64
    last = 99
    pf[last] = vtx.shape[0] - 1                          # runs past the end
    assert records.check(hdr, pf, vtx, 4, 64, 8) == (2, 3, 1)


def test_record_fields_round_trip_at_their_extremes():
    """Header bits 0-23 hold the light id and bits 24-31 the path length, the
    vertex weight is the float32 whose bits the record holds, and path p of a
    pixel starts after the pixel's earlier paths: checked with light ids up
    to 2^24 - 1, lengths up to 255 and weights that are not integers."""
    from oracle.records import unpack
    lights = np.array([0, 1, 0xFFFF, 0x10000, 0xABCDEF, 0xFFFFFF], dtype=np.uint32)
    lengths = np.array([0, 255, 1, 7, 2, 3], dtype=np.uint32)
    hdr = (lengths << 24) | lights
    spp = 3
    pix_first = np.array([5, 5 + int(lengths[:3].sum())], dtype=np.uint32)
    nv = 5 + int(lengths.sum())
    w = np.linspace(0.1, 0.9, nv).astype(np.float32)
    vtx = np.stack([np.arange(nv, dtype=np.uint32) * 7, w.view(np.uint32)], axis=1)
    L, light, first, texel, weight = unpack(hdr, pix_first, vtx, spp)
    assert L.tolist() == lengths.tolist() and light.tolist() == lights.tolist()
    assert first.tolist() == [5, 5, 260, 261, 268, 270]
    assert texel.tolist() == (np.arange(nv) * 7).tolist()
    assert np.array_equal(weight, w.astype(np.float64))
