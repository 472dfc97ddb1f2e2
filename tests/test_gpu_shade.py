"""GPU parity of encode / shade (both forms) / decode against the FP64 oracle.

Tolerance for XYZ and latent pixels: |x - x_ref| <= 2e-5 |x_ref| + 1e-7 per
component.  Every input is non-negative, so float32 sums and products carry
relative error (a few ulps times the term count) far below that bound.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import records as orec
from oracle import shade as osh
from tests.conftest import xyz_close
from tests.gpu_util import dev_f32, records_of_pixels, to_np

pytestmark = pytest.mark.gpu

REL, FLOOR = 2e-5, 1e-7


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd import ops as o
    return o


@pytest.fixture(scope="module")
def cfg0():
    return synth.workload(0)


def _paths(ops, hdr, pf, vtx, spp):
    return ops.Paths.from_numpy(hdr, pf, vtx, spp)


# ------------------------------------------------------------------ encode / decode

@pytest.mark.parametrize("k,n,m", [(6, 31, 64), (9, 31, 1000), (6, 31, 70001), (9, 81, 4099),
                                   (31, 31, 300), (48, 128, 129), (1, 5, 17)])
def test_encode_matches_oracle(ops, k, n, m):
    rng = np.random.default_rng(k * 1000 + n)
    E = rng.uniform(size=(k, n)).astype(np.float32)
    S = rng.uniform(size=(m, n)).astype(np.float32)
    Z = ops.encode(torch.from_numpy(E).cuda(), dev_f32(S), n=n)
    torch.cuda.synchronize()
    Zp = to_np(ops.from_blocked(Z, k))
    ref = osh.encode(E, S)
    assert xyz_close(Zp, ref, 1e-5, 1e-7) <= 1.0
    Zr = to_np(Z).reshape(m, -1, 4)
    assert (Zr[:, :, 3] == 0).all()  # the 4th float of every block is 0


def test_encode_writes_whole_padded_rows(ops, cfg0):
    Zpad = torch.full((64, 16), float("nan"), device="cuda")
    ops.encode(torch.from_numpy(cfg0["E"]).cuda(), dev_f32(cfg0["refl"]), n=31, out=Zpad)
    Z = to_np(Zpad)
    assert np.isfinite(Z).all() and (Z[:, 8:] == 0).all()


@pytest.mark.parametrize("k,n,npx", [(6, 31, 1000), (9, 81, 777), (33, 31, 300)])
def test_decode_matches_oracle(ops, k, n, npx):
    rng = np.random.default_rng(k + n)
    D = rng.uniform(size=(n, k)).astype(np.float32)
    T = synth.cmf_matrix(n)
    z = rng.uniform(size=(npx, k)).astype(np.float32)
    zb = ops.to_blocked(torch.from_numpy(z).cuda(), k)
    xyz, sp = ops.decode_xyz(torch.from_numpy(D).cuda(), torch.from_numpy(T).cuda(), zb, k,
                             spectra=True)
    torch.cuda.synchronize()
    s_ref, x_ref = osh.decode(D, T, z)
    assert xyz_close(to_np(xyz), x_ref, REL, FLOOR) <= 1.0
    assert xyz_close(to_np(sp), s_ref, REL, FLOOR) <= 1.0


# ------------------------------------------------------------------ config-0 frame in full

def test_cfg0_spectral_full_frame(ops, cfg0):
    hdr, pf, vtx = synth.gen_paths(cfg0["paths"])
    P = _paths(ops, hdr, pf, vtx, 1)
    xyz = ops.shade_spectral(P, dev_f32(cfg0["refl"]), dev_f32(cfg0["illum"]),
                             torch.from_numpy(cfg0["T"]).cuda(), 31)
    torch.cuda.synchronize()
    ref = osh.shade_spectral(hdr, pf, vtx, 1, cfg0["refl"], cfg0["illum"], cfg0["T"])
    assert xyz_close(to_np(xyz), ref, REL, FLOOR) <= 1.0


def test_cfg0_latent_end_to_end(ops, cfg0):
    """encode -> shade (fused B = 2 passes) -> decode on the GPU against the
    oracle's FP64 encode -> shade -> decode of the same float32 inputs."""
    hdr, pf, vtx = synth.gen_paths(cfg0["paths"])
    P = _paths(ops, hdr, pf, vtx, 1)
    E = torch.from_numpy(cfg0["E"]).cuda()
    D = torch.from_numpy(cfg0["D"]).cuda()
    T = torch.from_numpy(cfg0["T"]).cuda()
    codes = ops.encode(E, dev_f32(cfg0["refl"]), n=31)
    lcodes = ops.encode(E, dev_f32(cfg0["illum"]), n=31)
    zimg = ops.shade_latent(P, codes, lcodes, 6)
    xyz = ops.decode_xyz(D, T, zimg, 6)
    torch.cuda.synchronize()
    z_ref, x_ref = osh.render_latent_xyz(hdr, pf, vtx, 1, cfg0["refl"], cfg0["illum"], cfg0["E"],
                                         cfg0["D"], cfg0["T"])
    assert xyz_close(to_np(ops.from_blocked(zimg, 6)), z_ref, REL, FLOOR) <= 1.0
    assert xyz_close(to_np(xyz), x_ref, REL, FLOOR) <= 1.0


def test_passes_reassemble_bitwise(ops, cfg0):
    """B single-block launches ("RGB passes") write the same bits as the fused launch."""
    spec = synth.PathSpec(n_pixels=5000, spp=4, l_min=0, l_max=6, n_tex=64, n_illum=8, seed=21)
    hdr, pf, vtx = synth.gen_paths(spec)
    P = _paths(ops, hdr, pf, vtx, 4)
    rng = np.random.default_rng(1)
    for k in (6, 9):
        codes = ops.to_blocked(torch.from_numpy(rng.uniform(size=(64, k)).astype(np.float32)).cuda(), k)
        lc = ops.to_blocked(torch.from_numpy(rng.uniform(size=(8, k)).astype(np.float32)).cuda(), k)
        fused = ops.shade_latent(P, codes, lc, k)
        passes = torch.full_like(fused, float("nan"))
        for b in range(ops.blocks(k)):
            ops.shade_latent(P, codes, lc, k, block_first=b, block_count=1, out=passes)
        torch.cuda.synchronize()
        assert torch.equal(fused, passes)


# ------------------------------------------------------------------ shapes, spp, lengths, tails

@pytest.mark.parametrize("spp", [1, 3, 4, 16, 64, 100])
@pytest.mark.parametrize("k", [6, 9])
def test_latent_spp_and_ragged_tails(ops, spp, k):
    n_px = {1: 20011, 3: 3001, 4: 5003, 16: 1001, 64: 257, 100: 67}[spp]
    spec = synth.PathSpec(n_pixels=n_px, spp=spp, l_min=0, l_max=8, n_tex=500, n_illum=37, seed=spp)
    hdr, pf, vtx = synth.gen_paths(spec)
    rng = np.random.default_rng(spp * 7 + k)
    codes = rng.uniform(0.2, 1.2, size=(500, k)).astype(np.float32)
    lc = rng.uniform(size=(37, k)).astype(np.float32)
    P = _paths(ops, hdr, pf, vtx, spp)
    zimg = ops.shade_latent(P, ops.to_blocked(torch.from_numpy(codes).cuda(), k),
                            ops.to_blocked(torch.from_numpy(lc).cuda(), k), k)
    torch.cuda.synchronize()
    ref = osh.shade_latent(hdr, pf, vtx, spp, codes, lc)
    assert xyz_close(to_np(ops.from_blocked(zimg, k)), ref, REL, FLOOR) <= 1.0


@pytest.mark.parametrize("spp", [1, 3, 8, 16, 64, 100])
@pytest.mark.parametrize("n", [31, 81])
def test_spectral_spp_and_ragged_tails(ops, spp, n):
    n_px = {1: 20011, 3: 3001, 8: 2003, 16: 1001, 64: 257, 100: 67}[spp]
    spec = synth.PathSpec(n_pixels=n_px, spp=spp, l_min=0, l_max=8, n_tex=300, n_illum=40, seed=spp)
    hdr, pf, vtx = synth.gen_paths(spec)
    rng = np.random.default_rng(spp + n)
    refl = synth.reflectances(rng, n, 300)
    illum = synth.illuminant_table(rng, n, 20, 20)
    T = synth.cmf_matrix(n)
    P = _paths(ops, hdr, pf, vtx, spp)
    xyz = ops.shade_spectral(P, dev_f32(refl), dev_f32(illum), torch.from_numpy(T).cuda(), n)
    torch.cuda.synchronize()
    ref = osh.shade_spectral(hdr, pf, vtx, spp, refl, illum, T)
    assert xyz_close(to_np(xyz), ref, REL, FLOOR) <= 1.0


def test_large_light_table_read_from_global(ops):
    """1024 lights x 31 samples do not fit the LDS staging budget."""
    n = 31
    spec = synth.PathSpec(n_pixels=4000, spp=4, l_min=1, l_max=3, n_tex=100, n_illum=1024, seed=8)
    hdr, pf, vtx = synth.gen_paths(spec)
    rng = np.random.default_rng(8)
    refl = synth.reflectances(rng, n, 100)
    illum = synth.illuminant_table(rng, n, 512, 512)
    T = synth.cmf_matrix(n)
    P = _paths(ops, hdr, pf, vtx, 4)
    xyz = ops.shade_spectral(P, dev_f32(refl), dev_f32(illum), torch.from_numpy(T).cuda(), n)
    k = 48
    codes = rng.uniform(size=(100, k)).astype(np.float32)
    lc = rng.uniform(size=(1024, k)).astype(np.float32)
    zimg = ops.shade_latent(P, ops.to_blocked(torch.from_numpy(codes).cuda(), k),
                            ops.to_blocked(torch.from_numpy(lc).cuda(), k), k)
    torch.cuda.synchronize()
    assert xyz_close(to_np(xyz), osh.shade_spectral(hdr, pf, vtx, 4, refl, illum, T), REL, FLOOR) <= 1
    assert xyz_close(to_np(ops.from_blocked(zimg, k)), osh.shade_latent(hdr, pf, vtx, 4, codes, lc),
                     REL, FLOOR) <= 1


def _padded(a, ld, fill):
    """numpy (m, n) -> device float32 rows of stride ld, padding set to fill."""
    a = np.asarray(a, dtype=np.float32)
    out = np.full((a.shape[0], ld), fill, dtype=np.float32)
    out[:, :a.shape[1]] = a
    return torch.from_numpy(out).cuda()


# Light counts that put the light table in each place the spectral kernel can
# read it from: colour-weighted in LDS (3 float4 per light and chunk), plain in
# LDS, and global memory (LDS budget 16 KiB).
@pytest.mark.parametrize("n,n_illum", [(31, 8), (31, 60), (31, 600), (81, 5), (81, 40), (81, 300),
                                       (128, 8), (128, 20), (128, 100), (5, 3), (50, 30), (50, 200)])
def test_spectral_light_tables_and_nonfinite_padding(ops, n, n_illum):
    """Row padding past n (reflectance and light rows, strides beyond the
    padded width) holds NaN and inf; the result must not see it."""
    spec = synth.PathSpec(n_pixels=1500, spp=8, l_min=0, l_max=5, n_tex=200, n_illum=n_illum,
                          seed=n * 1000 + n_illum)
    hdr, pf, vtx = synth.gen_paths(spec)
    rng = np.random.default_rng(n + n_illum)
    refl = synth.reflectances(rng, n, 200)
    illum = synth.illuminant_table(rng, n, n_illum // 2, n_illum - n_illum // 2)
    T = synth.cmf_matrix(n)
    ld = 4 * ((n + 3) // 4) + 8
    P = _paths(ops, hdr, pf, vtx, 8)
    ref = osh.shade_spectral(hdr, pf, vtx, 8, refl, illum, T)
    for fill in (float("nan"), float("inf")):
        xyz = ops.shade_spectral(P, _padded(refl, ld, fill), _padded(illum, ld, fill),
                                 torch.from_numpy(T).cuda(), n)
        torch.cuda.synchronize()
        out = to_np(xyz)
        assert np.isfinite(out).all()
        assert xyz_close(out, ref, REL, FLOOR) <= 1.0


def test_identity_codec_latent_equals_spectral(ops, cfg0):
    """k = n = 31 (padded to 33) with E = D = I: the latent XYZ equals the
    spectral oracle's XYZ within the tolerance."""
    spec = synth.PathSpec(n_pixels=3000, spp=4, l_min=0, l_max=4, n_tex=64, n_illum=8, seed=4)
    hdr, pf, vtx = synth.gen_paths(spec)
    P = _paths(ops, hdr, pf, vtx, 4)
    k = 31
    E = np.eye(31, dtype=np.float32)
    D = np.eye(31, dtype=np.float32)
    Et, Dt = torch.from_numpy(E).cuda(), torch.from_numpy(D).cuda()
    T = torch.from_numpy(cfg0["T"]).cuda()
    codes = ops.encode(Et, dev_f32(cfg0["refl"]), n=31)
    lc = ops.encode(Et, dev_f32(cfg0["illum"]), n=31)
    xyz = ops.decode_xyz(Dt, T, ops.shade_latent(P, codes, lc, k), k)
    torch.cuda.synchronize()
    ref = osh.shade_spectral(hdr, pf, vtx, 4, cfg0["refl"], cfg0["illum"], cfg0["T"])
    assert xyz_close(to_np(xyz), ref, REL, FLOOR) <= 1.0


def test_empty_and_lightonly_frames(ops, cfg0):
    empty = ops.Paths(torch.zeros(0, dtype=torch.int32, device="cuda"),
                      torch.zeros(0, dtype=torch.int32, device="cuda"),
                      torch.zeros(0, 2, dtype=torch.int32, device="cuda"), 0, 4)
    codes = dev_f32(np.ones((4, 8), dtype=np.float32))
    assert ops.shade_latent(empty, codes, codes, 6).shape == (0, 8)
    # every path sees the light directly (L = 0): no vertex records at all
    spec = synth.PathSpec(n_pixels=100, spp=2, l_min=0, l_max=0, n_tex=64, n_illum=8, seed=2)
    hdr, pf, vtx = synth.gen_paths(spec)
    assert vtx.shape[0] == 0
    P = _paths(ops, hdr, pf, vtx, 2)
    xyz = ops.shade_spectral(P, dev_f32(cfg0["refl"]), dev_f32(cfg0["illum"]),
                             torch.from_numpy(cfg0["T"]).cuda(), 31)
    torch.cuda.synchronize()
    ref = osh.shade_spectral(hdr, pf, vtx, 2, cfg0["refl"], cfg0["illum"], cfg0["T"])
    assert xyz_close(to_np(xyz), ref, REL, FLOOR) <= 1.0


# ------------------------------------------------------------------ records

def test_check_paths_counts_exactly(ops):
    spec = synth.PathSpec(n_pixels=3000, spp=4, l_min=1, l_max=4, n_tex=64, n_illum=8, seed=13)
    hdr, pf, vtx = synth.gen_paths(spec)
    hdr, pf, vtx = hdr.copy(), pf.copy(), vtx.copy()
    rng = np.random.default_rng(0)
    hdr[rng.choice(hdr.size, 17, replace=False)] |= 0xFFFF   # light ids >= 8
    vtx[rng.choice(vtx.shape[0], 23, replace=False), 0] = 64 + rng.integers(0, 5, 23).astype(np.uint32)
    pf[[5, 2999]] = vtx.shape[0] - 1                          # ranges past the end
    P = _paths(ops, hdr, pf, vtx, 4)
    got = tuple(int(x) for x in to_np(ops.check_paths(P, 64, 8)))
    assert got == orec.check(hdr, pf, vtx, 4, 64, 8)
    assert got[0] >= 17 and got[2] >= 1


def test_malformed_records_stay_in_bounds(ops, cfg0):
    """Out-of-range ids are clamped: the kernels finish and write finite values."""
    spec = synth.PathSpec(n_pixels=500, spp=4, l_min=1, l_max=4, n_tex=64, n_illum=8, seed=14)
    hdr, pf, vtx = synth.gen_paths(spec)
    hdr, pf, vtx = hdr.copy(), pf.copy(), vtx.copy()
    hdr[::7] |= 0xFFFFFF
    vtx[::5, 0] = 0xFFFFFFF0
    pf[-3:] = vtx.shape[0] - 2
    P = _paths(ops, hdr, pf, vtx, 4)
    xyz = ops.shade_spectral(P, dev_f32(cfg0["refl"]), dev_f32(cfg0["illum"]),
                             torch.from_numpy(cfg0["T"]).cuda(), 31)
    codes = ops.encode(torch.from_numpy(cfg0["E"]).cuda(), dev_f32(cfg0["refl"]), n=31)
    z = ops.shade_latent(P, codes, codes[:8], 6)
    torch.cuda.synchronize()
    assert torch.isfinite(xyz).all() and torch.isfinite(z).all()


# The last three put more records in a wavefront's round than its LDS map
# holds (2048) in some or all rounds, so both ways of making records run.
@pytest.mark.parametrize("n_pixels,spp,l_min,l_max", [(777, 16, 1, 8), (1000, 1, 1, 4), (333, 3, 0, 2),
                                                      (129, 64, 1, 8), (65, 100, 0, 5), (40, 130, 2, 2),
                                                      (50, 64, 30, 60), (300, 8, 20, 40), (90, 130, 0, 40)])
def test_device_generator_matches_synth(ops, n_pixels, spp, l_min, l_max):
    spec = synth.PathSpec(n_pixels=n_pixels, spp=spp, l_min=l_min, l_max=l_max, n_tex=1 << 20,
                          n_illum=256, seed=77 + spp)
    hdr, pf, vtx = synth.gen_paths(spec)
    P = ops.gen_paths(n_pixels, spp, l_min, l_max, 1 << 20, 256, 77 + spp)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(P.hdr).view(np.uint32), hdr)
    assert np.array_equal(to_np(P.pix_first).view(np.uint32), pf)
    assert np.array_equal(to_np(P.vtx).view(np.uint32), vtx)
    idx = to_np(ops.gen_indices(5, 10000, 12345, ctr0=3)).view(np.uint32)
    assert np.array_equal(idx, synth.uniform_indices(5, 3, 10000, 12345))


# ------------------------------------------------------------------ frame scale (config 1)

@pytest.mark.slow
def test_cfg1_frame_sampled_pixels(ops):
    """1920x1080 at 16 spp, L in 1..4, 1024^2 x 31 texture: the whole frame is
    shaded on the GPU in the configuration the benchmark times; 65,536
    seeded pixels are checked against the oracle, spectral and latent."""
    w = synth.workload(1)
    spec = w["paths"]
    P = ops.gen_paths(spec.n_pixels, spec.spp, spec.l_min, spec.l_max, spec.n_tex, spec.n_illum,
                      spec.seed)
    refl, illum, T = dev_f32(w["refl"]), dev_f32(w["illum"]), torch.from_numpy(w["T"]).cuda()
    E, D = torch.from_numpy(w["E"]).cuda(), torch.from_numpy(w["D"]).cuda()
    xyz_s = ops.shade_spectral(P, refl, illum, T, 31)
    codes = ops.encode(E, refl, n=31)
    lc = ops.encode(E, illum, n=31)
    zimg = ops.shade_latent(P, codes, lc, 6)
    xyz_l = ops.decode_xyz(D, T, zimg, 6)
    torch.cuda.synchronize()
    pix = np.sort(np.random.default_rng(1).choice(spec.n_pixels, 65536, replace=False))
    hdr, pf, vtx = records_of_pixels(spec, pix)
    ref_s = osh.shade_spectral(hdr, pf, vtx, spec.spp, w["refl"], w["illum"], w["T"])
    assert xyz_close(to_np(xyz_s)[pix], ref_s, REL, FLOOR) <= 1.0
    _, ref_l = osh.render_latent_xyz(hdr, pf, vtx, spec.spp, w["refl"], w["illum"], w["E"], w["D"],
                                     w["T"])
    assert xyz_close(to_np(xyz_l)[pix], ref_l, REL, FLOOR) <= 1.0
