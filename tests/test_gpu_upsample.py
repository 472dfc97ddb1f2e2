"""GPU upsampling network (Sec. 5) against the FP64 oracle.

Tolerance, derived from the arithmetic (per output channel c of texel i):
the fp16 path rounds W2, h1, W3 and h2 to fp16 (unit roundoff u16 = 2^-11)
and accumulates in fp32; a 128-term fp32 sum adds at most g = 130 * 2^-24
relative to the sum of |terms|; the activations are fp32 (within
ua = 8 * 2^-24 relative).  With S2_j = sum_i |W2_ji| |h1_i| and silu's
Lipschitz constant 1.1:
    e(p2_j) <= (2 u16 + g + ua) S2_j + g |b2_j|
    e(h2_j) <= 1.1 e(p2_j) + ua |h2_j|
    e(z_c)  <= sum_j |W3_cj| e(h2_j) + (2 u16 + g) sum_j |W3_cj| |h2_j| + g |b3_c|
The fp32 path has u16 = 0.  The fp16 kernel carries s = -h / ln 2 between layers
(-log2 e folded into the layer-1 weights and the biases in fp32, -ln 2 applied in
the output FMA): each fold is one more fp32 rounding, a few 2^-24 relative, inside
the slack of g and ua; rounding s to fp16 is the same relative u16 as rounding h.
Checked element by element against this bound.
"""

import numpy as np
import pytest
import torch

from oracle import upsample as ou

pytestmark = pytest.mark.gpu

U16, G, UA = 2.0 ** -11, 130 * 2.0 ** -24, 8 * 2.0 ** -24


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd import ops as o
    return o


def _net(k, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    h = 128
    net = dict(W1=rng.normal(0, 2.0 * scale, (h, 3)), b1=rng.normal(0, 0.5, h),
               W2=rng.normal(0, scale / np.sqrt(h), (h, h)), b2=rng.normal(0, 0.5, h),
               W3=rng.normal(0, scale / np.sqrt(h), (k, h)), b3=rng.normal(0, 0.5, k))
    return {key: v.astype(np.float32) for key, v in net.items()}


def _bound(net, rgb, u16):
    f = {key: np.asarray(v, np.float64) for key, v in net.items()}
    h1, h2 = ou.mlp_hidden(net, rgb)
    S2 = np.abs(h1) @ np.abs(f["W2"]).T
    ep2 = (2 * u16 + G + UA) * S2 + G * np.abs(f["b2"])
    eh2 = 1.1 * ep2 + UA * np.abs(h2)
    A3 = np.abs(f["W3"])
    return eh2 @ A3.T + (2 * u16 + G) * (np.abs(h2) @ A3.T) + G * np.abs(f["b3"])


def _blocked_to_k(z, k):
    c = np.arange(k)
    return z[:, 4 * (c // 3) + c % 3]


@pytest.mark.parametrize("precision", ["f16", "f32"])
@pytest.mark.parametrize("k,m", [(6, 16 * 4 * 37 + 5), (9, 1), (3, 16), (16, 333), (17, 1000),
                                 (31, 257), (48, 2049)])
def test_upsample_matches_oracle_within_derived_bound(ops, precision, k, m):
    net = _net(k, seed=k)
    rgb = np.random.default_rng(100 + k).uniform(0, 1, (m, 3)).astype(np.float32)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    z = ops.upsample({key: t(v) for key, v in net.items()}, t(rgb), k, precision=precision)
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    ref = ou.upsample(net, rgb)
    bound = _bound(net, rgb, U16 if precision == "f16" else 0.0)
    err = np.abs(_blocked_to_k(z, k).astype(np.float64) - ref)
    assert (err <= bound).all(), float((err / bound).max())
    # the bound is not vacuous: errors use a visible part of it in fp16
    if precision == "f16" and m > 100:
        assert (err / bound).max() > 1e-3
    # padding of the blocked layout is zero
    nb = (k + 2) // 3
    cols = [c for c in range(z.shape[1]) if c % 4 == 3 or c // 4 >= nb or 3 * (c // 4) + c % 4 >= k]
    assert (z[:, cols] == 0).all()


@pytest.mark.parametrize("precision", ["f16", "f32"])
def test_upsample_full_texture_sampled_rows(ops, precision):
    """The 4096^2-texel RGBA texture of the throughput measurement, in the
    same launch: 8192 sampled rows (and the first and last) against the
    oracle within the derived bound."""
    k, side = 6, 4096
    net = _net(k, seed=11)
    rng = np.random.default_rng(12)
    rgba = rng.uniform(0, 1, (side * side, 4)).astype(np.float32)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    out = torch.empty(side * side, 8, device="cuda")
    ops.upsample({key: t(v) for key, v in net.items()}, t(rgba), k, precision=precision, out=out)
    rows = np.concatenate([[0, side * side - 1], rng.choice(side * side, 8192, replace=False)])
    z = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    rgb = rgba[rows, :3]
    bound = _bound(net, rgb, U16 if precision == "f16" else 0.0)
    assert (np.abs(_blocked_to_k(z, k).astype(np.float64) - ou.upsample(net, rgb)) <= bound).all()


def test_upsample_strided_input_and_wide_output(ops):
    """rgb rows with stride 4 (RGBA) and an output stride wider than needed."""
    k, m = 6, 1000
    net = _net(k, seed=1)
    rgba = np.random.default_rng(2).uniform(0, 1, (m, 4)).astype(np.float32)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    out = torch.full((m, 16), 7.0, device="cuda")
    ops.upsample({key: t(v) for key, v in net.items()}, t(rgba), k, precision="f32", out=out)
    torch.cuda.synchronize()
    z = out.cpu().numpy()
    ref = ou.upsample(net, rgba[:, :3])
    assert (np.abs(_blocked_to_k(z, k) - ref) <= _bound(net, rgba[:, :3], 0.0)).all()
    assert (z[:, 8:] == 0).all() and (z[:, [3, 7]] == 0).all()


def test_upsample_empty_and_deterministic(ops):
    k = 9
    net = _net(k, seed=3)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    dnet = {key: t(v) for key, v in net.items()}
    empty = ops.upsample(dnet, torch.zeros(0, 3, device="cuda"), k)
    assert empty.shape == (0, 12)
    rgb = t(np.random.default_rng(4).uniform(0, 1, (50000, 3)).astype(np.float32))
    a = ops.upsample(dnet, rgb, k)
    b = ops.upsample(dnet, rgb, k)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_upsampled_codes_shade_like_encoded_ones(ops):
    """Codes from the network feed hc_shade_latent directly: a frame shaded
    with upsampled texels equals the oracle's latent frame on those codes."""
    from oracle import shade as osh
    import synth
    k, n_tex = 6, 4096
    net = _net(k, seed=5, scale=0.5)
    rgb = np.random.default_rng(6).uniform(0, 1, (n_tex, 3)).astype(np.float32)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    codes = ops.upsample({key: t(v) for key, v in net.items()}, t(rgb), k, precision="f32")
    spec = synth.PathSpec(n_pixels=4096, spp=4, l_min=1, l_max=3, n_tex=n_tex, n_illum=8, seed=9)
    hdr, pf, vtx = synth.gen_paths(spec)
    lc = np.abs(np.random.default_rng(7).normal(size=(8, k))).astype(np.float32)
    P = ops.Paths.from_numpy(hdr, pf, vtx, spec.spp)
    z = ops.shade_latent(P, codes, ops.to_blocked(t(lc), k), k)
    torch.cuda.synchronize()
    got = ops.from_blocked(z, k).cpu().numpy()
    zc = _blocked_to_k(codes.cpu().numpy(), k)
    want = osh.shade_latent(hdr, pf, vtx, spec.spp, zc, lc)
    # codes from the network may be negative: the bound scales with the mean
    # of the absolute per-path products
    scale = osh.shade_latent(hdr, pf, vtx, spec.spp, np.abs(zc), lc)
    assert (np.abs(got - want) <= 2e-5 * scale + 1e-7).all()
