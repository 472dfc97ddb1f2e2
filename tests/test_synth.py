"""The seeded generators: determinism, ranges, the counter-based path
generator's self-consistency and the colour-matching fit's known integrals."""

import numpy as np

import synth


def test_cmf_fit_equal_energy_integrals():
    """The CIE 1931 functions integrate to ~106.86 each over the visible
    range (equal-energy white has x = y = z = 1/3); the multi-lobe fit keeps
    that to about 0.1 %."""
    lam = np.arange(360.0, 831.0, 1.0)
    ints = synth.cmf_fit_cie1931(lam).sum(axis=1)
    assert np.allclose(ints, 106.86, rtol=2e-3)


def test_cmf_matrix_normalises_equal_energy_y():
    for n in (31, 81):
        T = synth.cmf_matrix(n)
        assert T.shape == (3, n)
        assert abs(float(T[1].astype(np.float64).sum()) - 1.0) < 1e-6


def test_workloads_are_deterministic():
    a, b = synth.workload(0), synth.workload(0)
    for key in ("refl", "illum", "E", "D", "T"):
        assert np.array_equal(a[key], b[key])
    assert a["refl"].shape == (64, 31) and a["illum"].shape == (8, 31)
    assert 0 <= a["refl"].min() and a["refl"].max() <= 1
    assert np.allclose(a["illum"].max(axis=1), 1.0)


def test_texture_is_a_convex_blend():
    w = synth.workload(1, texture_side=64)
    assert w["refl"].shape == (4096, 31)
    assert w["refl"].min() >= 0 and w["refl"].max() <= 1
    wts = synth.perlin_weights(1001, 64)
    assert np.allclose(wts.sum(axis=1), 1.0)


def test_paths_layout_and_ranges():
    spec = synth.PathSpec(n_pixels=1000, spp=4, l_min=1, l_max=4, n_tex=1 << 20, n_illum=32, seed=7)
    hdr, pf, vtx = synth.gen_paths(spec)
    L = (hdr >> 24).astype(np.int64)
    assert L.min() == 1 and L.max() == 4
    assert (hdr & 0xFFFFFF).max() < 32
    assert pf[0] == 0 and np.array_equal(np.diff(pf.astype(np.int64)), L.reshape(1000, 4).sum(1)[:-1])
    assert vtx.shape[0] == L.sum() and vtx[:, 0].max() < 1 << 20
    w = vtx[:, 1].view(np.float32)
    assert w.min() >= 0 and w.max() < 1
    assert abs(L.mean() - 2.5) < 0.1


def test_sampled_paths_match_the_whole_frame():
    spec = synth.PathSpec(n_pixels=500, spp=16, l_min=1, l_max=8, n_tex=4096, n_illum=256, seed=3)
    hdr, pf, vtx = synth.gen_paths(spec, chunk_pixels=64)
    pick = np.array([0, 1, 17, 4000, 7999])
    L, light, tex, wt = synth.path_records(spec, pick)
    assert np.array_equal(L, hdr[pick] >> 24) and np.array_equal(light, hdr[pick] & 0xFFFFFF)
    Lall = (hdr >> 24).astype(np.int64)
    within = np.cumsum(Lall.reshape(500, 16), axis=1) - Lall.reshape(500, 16)
    first = (pf.astype(np.int64)[:, None] + within).ravel()
    for i, p in enumerate(pick):
        j = first[p]
        assert np.array_equal(tex[i, :L[i]], vtx[j:j + L[i], 0])
        assert np.array_equal(wt[i, :L[i]].view(np.uint32), vtx[j:j + L[i], 1])


def test_mix64_is_a_bijection_sample():
    x = np.arange(1 << 16, dtype=np.uint64)
    assert np.unique(synth.mix64(x)).size == x.size
    assert synth.mix64(np.uint64(0)) == 0


def test_chain_records_layout():
    from oracle.records import unpack
    C, bounces = 5, 3
    hdr, pf, vtx = synth.chain_records(C, bounces)
    length, light, first, texel, weight = unpack(hdr, pf, vtx, 1)
    assert length.tolist() == [b for b in range(bounces + 1) for _ in range(C)]
    assert light.tolist() == list(range(C)) * (bounces + 1)
    assert (weight == 1.0).all() and vtx.shape[0] == C * (0 + 1 + 2 + 3)
    for p in range(hdr.size):
        b, c = divmod(p, C)
        assert texel[first[p]:first[p] + b].tolist() == [c * bounces + v for v in range(b)]
