"""The latent frame in one launch (hc_shade_latent_xyz, Eq. 6 products with
the per-pixel decode of Eq. 4 in the epilogue) and its decoder matrix
(hc_decode_matrix, M = T D).

* M against the oracle's decode of unit codes (column c of M is the XYZ of
  the code e_c), zero past k;
* the fused frame bit for bit against hc_shade_latent followed by
  hc_decode_xyz (the same pixel means and the same dot with the same M);
* the fused frame against the oracle's FP64 shade -> decode within the
  shading tolerance |x - x_ref| <= 2e-5 |x_ref| + 1e-7 (all inputs are
  non-negative, so float32 sums carry relative error far below it).
"""

import numpy as np
import pytest
import torch

import synth
from oracle import shade as osh
from tests.conftest import xyz_close
from tests.gpu_util import dev_f32, to_np

pytestmark = pytest.mark.gpu

REL, FLOOR = 2e-5, 1e-7


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd import ops as o
    return o


def _codec(rng, k, n):
    D = rng.uniform(size=(n, k)).astype(np.float32)
    T = synth.cmf_matrix(n)
    return D, T, torch.from_numpy(D).cuda(), torch.from_numpy(T).cuda()


@pytest.mark.parametrize("k,n", [(1, 5), (6, 31), (9, 81), (31, 31), (47, 128), (48, 128)])
def test_decode_matrix_is_the_decode_of_unit_codes(ops, k, n):
    rng = np.random.default_rng(10 * k + n)
    D, T, Dt, Tt = _codec(rng, k, n)
    M = ops.decode_matrix(Dt, Tt, k)
    torch.cuda.synchronize()
    assert tuple(M.shape) == (3, 3 * ops.blocks(k))
    Mn = to_np(M)
    _, x_unit = osh.decode(D, T, np.eye(k))  # row c: XYZ of the unit code e_c
    assert xyz_close(Mn[:, :k], x_unit.T, REL, FLOOR) <= 1.0
    assert (Mn[:, k:] == 0).all()


def _frame(ops, rng, spec, k):
    hdr, pf, vtx = synth.gen_paths(spec)
    P = ops.Paths.from_numpy(hdr, pf, vtx, spec.spp)
    codes = rng.uniform(0.2, 1.2, size=(spec.n_tex, k)).astype(np.float32)
    lc = rng.uniform(size=(spec.n_illum, k)).astype(np.float32)
    cb = ops.to_blocked(torch.from_numpy(codes).cuda(), k)
    lb = ops.to_blocked(torch.from_numpy(lc).cuda(), k)
    return (hdr, pf, vtx), P, codes, lc, cb, lb


def _xyz_ref(rec, spp, codes, lc, D, T):
    """The oracle's shade -> decode.  For k not a multiple of 3 the codes
    and D get zero channels up to 3B (the blockwise product needs whole
    triplets; zero columns of D leave the decode unchanged)."""
    k = codes.shape[1]
    pad = -k % 3
    if pad:
        codes, lc = (np.pad(a, ((0, 0), (0, pad))) for a in (codes, lc))
        D = np.pad(D, ((0, 0), (0, pad)))
    return osh.decode(D, T, osh.shade_latent(*rec, spp, codes, lc))[1]


def _both_routes(ops, P, cb, lb, Dt, Tt, k):
    two = ops.decode_xyz(Dt, Tt, ops.shade_latent(P, cb, lb, k), k)
    one = ops.shade_latent_xyz(P, cb, lb, ops.decode_matrix(Dt, Tt, k), k)
    torch.cuda.synchronize()
    return one, two


@pytest.mark.parametrize("spp", [1, 3, 16, 100])
@pytest.mark.parametrize("k", [1, 6, 9, 31, 48])
def test_fused_frame_equals_shade_then_decode(ops, k, spp):
    n_px = {1: 20011, 3: 3001, 16: 1001, 100: 67}[spp]
    spec = synth.PathSpec(n_pixels=n_px, spp=spp, l_min=0, l_max=8, n_tex=500, n_illum=37, seed=spp + k)
    rng = np.random.default_rng(spp * 100 + k)
    (hdr, pf, vtx), P, codes, lc, cb, lb = _frame(ops, rng, spec, k)
    D, T, Dt, Tt = _codec(rng, k, 31)
    one, two = _both_routes(ops, P, cb, lb, Dt, Tt, k)
    assert torch.equal(one, two)
    x_ref = _xyz_ref((hdr, pf, vtx), spp, codes, lc, D, T)
    assert xyz_close(to_np(one), x_ref, REL, FLOOR) <= 1.0


def test_fused_frame_with_lights_in_global_memory(ops):
    """1024 light codes of k = 48 do not fit the LDS budget: the decoder
    matrix is then the whole of the staged LDS."""
    k = 48
    spec = synth.PathSpec(n_pixels=4000, spp=4, l_min=0, l_max=3, n_tex=100, n_illum=1024, seed=8)
    rng = np.random.default_rng(8)
    (hdr, pf, vtx), P, codes, lc, cb, lb = _frame(ops, rng, spec, k)
    D, T, Dt, Tt = _codec(rng, k, 64)
    one, two = _both_routes(ops, P, cb, lb, Dt, Tt, k)
    assert torch.equal(one, two)
    x_ref = _xyz_ref((hdr, pf, vtx), 4, codes, lc, D, T)
    assert xyz_close(to_np(one), x_ref, REL, FLOOR) <= 1.0


def test_fused_frame_config0_end_to_end():
    """encode -> decoder matrix -> fused frame against the oracle's FP64
    encode -> shade -> decode (Fig. 2b) on the small frame in full."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd import ops
    cfg0 = synth.workload(0)
    hdr, pf, vtx = synth.gen_paths(cfg0["paths"])
    P = ops.Paths.from_numpy(hdr, pf, vtx, 1)
    E = torch.from_numpy(cfg0["E"]).cuda()
    M = ops.decode_matrix(torch.from_numpy(cfg0["D"]).cuda(), torch.from_numpy(cfg0["T"]).cuda(), 6)
    xyz = ops.shade_latent_xyz(P, ops.encode(E, dev_f32(cfg0["refl"]), n=31),
                               ops.encode(E, dev_f32(cfg0["illum"]), n=31), M, 6)
    torch.cuda.synchronize()
    _, x_ref = osh.render_latent_xyz(hdr, pf, vtx, 1, cfg0["refl"], cfg0["illum"], cfg0["E"], cfg0["D"],
                                     cfg0["T"])
    assert xyz_close(to_np(xyz), x_ref, REL, FLOOR) <= 1.0


def test_fused_frame_over_a_table_past_the_cache(ops):
    """6,000,000 texels of k = 9 (288 MB, past the 256 MB cache) take the
    launch shape for HBM-resident tables, whose LDS reservation also holds
    the light codes and the decoder matrix."""
    k, n_tex = 9, 6_000_000
    spec = synth.PathSpec(n_pixels=20000, spp=4, l_min=1, l_max=8, n_tex=n_tex, n_illum=16, seed=31)
    hdr, pf, vtx = synth.gen_paths(spec)
    P = ops.Paths.from_numpy(hdr, pf, vtx, 4)
    rng = np.random.default_rng(31)
    codes = rng.uniform(0.5, 1.5, size=(n_tex, k)).astype(np.float32)
    lc = rng.uniform(size=(16, k)).astype(np.float32)
    cb = ops.to_blocked(torch.from_numpy(codes).cuda(), k)
    assert cb.numel() * 4 > 256 * 2 ** 20
    lb = ops.to_blocked(torch.from_numpy(lc).cuda(), k)
    D, T, Dt, Tt = _codec(rng, k, 81)
    one, two = _both_routes(ops, P, cb, lb, Dt, Tt, k)
    assert torch.equal(one, two)
    x_ref = _xyz_ref((hdr, pf, vtx), 4, codes, lc, D, T)
    assert xyz_close(to_np(one), x_ref, REL, FLOOR) <= 1.0


def test_fused_frame_empty_and_light_only(ops):
    empty = ops.Paths(torch.zeros(0, dtype=torch.int32, device="cuda"),
                      torch.zeros(0, dtype=torch.int32, device="cuda"),
                      torch.zeros(0, 2, dtype=torch.int32, device="cuda"), 0, 4)
    codes = dev_f32(np.ones((4, 8), dtype=np.float32))
    M = torch.zeros(3, 6, device="cuda")
    assert ops.shade_latent_xyz(empty, codes, codes, M, 6).shape == (0, 3)
    # L = 0 everywhere: no vertex records, each pixel is the decoded light code
    k = 6
    spec = synth.PathSpec(n_pixels=100, spp=2, l_min=0, l_max=0, n_tex=64, n_illum=8, seed=2)
    rng = np.random.default_rng(2)
    (hdr, pf, vtx), P, codes, lc, cb, lb = _frame(ops, rng, spec, k)
    assert vtx.shape[0] == 0
    D, T, Dt, Tt = _codec(rng, k, 31)
    one, two = _both_routes(ops, P, cb, lb, Dt, Tt, k)
    assert torch.equal(one, two)
    x_ref = _xyz_ref((hdr, pf, vtx), 2, codes, lc, D, T)
    assert xyz_close(to_np(one), x_ref, REL, FLOOR) <= 1.0
