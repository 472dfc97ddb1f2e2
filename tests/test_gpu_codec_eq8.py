"""GPU codec step with the four-term objective of Eq. 8 against the oracle.

Same bars as the two-term step: float32 loss within 1e-5 relative, gradients
per element |g - g_ref| <= 1e-4 max(|g_ref|, 1e-3 |g_ref|_inf) and normwise
1e-4; the float64 instance within 1e-10 of the oracle and 1e-7 of central
finite differences of the oracle's loss.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import codec as oc
from tests.gpu_util import box_codec, to_np

pytestmark = pytest.mark.gpu

W = (0.5, 0.75, 1.0, 0.5)


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd import ops as o
    return o


def _grad_ok(g, ref, rel=1e-4, scale=None):
    g, ref = np.asarray(g, np.float64), np.asarray(ref, np.float64)
    floor = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    if scale is not None:
        floor = np.maximum(floor, scale)
    elem = (np.abs(g - ref) <= rel * floor).all()
    norm = np.linalg.norm(g - ref) <= rel * np.linalg.norm(ref)
    return bool(elem and norm)


def _pairs(n, N, seed):
    rng = np.random.default_rng(seed)
    return (synth.reflectances(rng, n, N),
            synth.illuminant_table(rng, n, N // 2, N - N // 2))


def _t(x, dt=np.float32):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dt))).cuda()


@pytest.mark.parametrize("n,k", [(31, 6), (31, 9), (81, 9), (81, 6), (31, 31)])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_eq8_loss_and_gradient_fp32(ops, n, k, seed):
    N = 65536 if seed == 0 else 4099
    rng = np.random.default_rng(seed)
    we, wd = synth.codec_init(rng, k, n)
    A, B = _pairs(n, N, 100 + seed)
    T = synth.cmf_matrix(n)
    ge = torch.empty(k, n, device="cuda")
    gd = torch.empty(n, k, device="cuda")
    loss = ops.codec_step(_t(we), _t(wd), _t(A), _t(B), N, grad_e=ge, grad_d=gd, objective="eq8",
                          T=_t(T), weights=W)
    torch.cuda.synchronize()
    L, rge, rgd = oc.loss_eq8_and_grad(we, wd, A, B, T, W)
    assert abs(float(loss) - L) <= 1e-5 * L
    assert _grad_ok(to_np(ge), rge) and _grad_ok(to_np(gd), rgd)


@pytest.mark.parametrize("n,k", [(81, 9), (81, 6), (31, 6)])
def test_eq8_near_fit_fp32(ops, n, k):
    """A near-fit codec (box filters), where each gradient element is a sum
    of per-pair terms of both signs much larger than the sum: per element
    |g - g_ref| <= 1e-4 max(|g_ref|, 1e-3 |g_ref|_inf, m) with m the sum of
    the terms' magnitudes (over 16-pair chunks; the error of a floating-point
    sum is bounded through the magnitudes of its terms), normwise 1e-4."""
    N = 8192
    we, wd = (w.astype(np.float32) for w in box_codec(k, n))
    A, B = _pairs(n, N, 77)
    T = synth.cmf_matrix(n)
    ge = torch.empty(k, n, device="cuda")
    gd = torch.empty(n, k, device="cuda")
    loss = ops.codec_step(_t(we), _t(wd), _t(A), _t(B), N, grad_e=ge, grad_d=gd, objective="eq8",
                          T=_t(T), weights=W)
    torch.cuda.synchronize()
    L, rge, rgd = oc.loss_eq8_and_grad(we, wd, A, B, T, W)
    me = md = 0.0
    for c in range(0, N, 16):
        _, ge_c, gd_c = oc.loss_eq8_and_grad(we, wd, A[c:c + 16], B[c:c + 16], T, W)
        me, md = me + np.abs(ge_c) * 16 / N, md + np.abs(gd_c) * 16 / N
    assert abs(float(loss) - L) <= 1e-5 * L
    assert _grad_ok(to_np(ge), rge, scale=me) and _grad_ok(to_np(gd), rgd, scale=md)


@pytest.mark.parametrize("n,k", [(81, 9), (81, 6), (31, 6)])
@pytest.mark.parametrize("weights", [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)])
def test_eq8_each_term_fp32(ops, n, k, weights):
    """Each term alone on the float32 kernels (the n = 81 one forms the
    code-space gradients of every term through D^T D), at the float32 bounds."""
    N = 4099
    rng = np.random.default_rng(31 + n + k)
    we, wd = synth.codec_init(rng, k, n)
    A, B = _pairs(n, N, 32 + n)
    T = synth.cmf_matrix(n)
    ge = torch.empty(k, n, device="cuda")
    gd = torch.empty(n, k, device="cuda")
    loss = ops.codec_step(_t(we), _t(wd), _t(A), _t(B), N, grad_e=ge, grad_d=gd, objective="eq8",
                          T=_t(T), weights=weights)
    torch.cuda.synchronize()
    L, rge, rgd = oc.loss_eq8_and_grad(we, wd, A, B, T, weights)
    assert abs(float(loss) - L) <= 1e-5 * L
    assert _grad_ok(to_np(ge), rge) and _grad_ok(to_np(gd), rgd)


@pytest.mark.parametrize("weights", [W, (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1),
                                     (2.0, 0.5, 0.25, 1.0)])
def test_eq8_each_term_fp64(ops, weights):
    """Each term alone, and another mix, in float64 against the oracle."""
    n, k, N = 31, 6, 777
    rng = np.random.default_rng(21)
    we, wd = (x.astype(np.float64) for x in synth.codec_init(rng, k, n))
    A, B = (x.astype(np.float64) for x in _pairs(n, N, 22))
    T = synth.cmf_matrix(n).astype(np.float64)
    d = np.float64
    ge = torch.empty(k, n, dtype=torch.float64, device="cuda")
    gd = torch.empty(n, k, dtype=torch.float64, device="cuda")
    loss = ops.codec_step(_t(we, d), _t(wd, d), _t(A, d), _t(B, d), N, grad_e=ge, grad_d=gd,
                          objective="eq8", T=_t(T, d), weights=weights)
    torch.cuda.synchronize()
    L, rge, rgd = oc.loss_eq8_and_grad(we, wd, A, B, T, weights)
    assert abs(float(loss) - L) <= 1e-12 * L
    assert np.allclose(to_np(ge), rge, rtol=1e-10, atol=1e-13 * max(np.abs(rge).max(), 1e-300))
    assert np.allclose(to_np(gd), rgd, rtol=1e-10, atol=1e-13 * max(np.abs(rgd).max(), 1e-300))


@pytest.mark.parametrize("seed", range(8))
def test_eq8_fp64_gradient_matches_oracle_and_finite_differences(ops, seed):
    n, k, N = (31, 6, 512) if seed % 2 == 0 else (81, 9, 300)
    rng = np.random.default_rng(400 + seed)
    we, wd = (x.astype(np.float64) for x in synth.codec_init(rng, k, n))
    A, B = (x.astype(np.float64) for x in _pairs(n, N, 500 + seed))
    T = synth.cmf_matrix(n).astype(np.float64)
    d = np.float64
    ge = torch.empty(k, n, dtype=torch.float64, device="cuda")
    gd = torch.empty(n, k, dtype=torch.float64, device="cuda")
    loss = ops.codec_step(_t(we, d), _t(wd, d), _t(A, d), _t(B, d), N, grad_e=ge, grad_d=gd,
                          objective="eq8", T=_t(T, d), weights=W)
    torch.cuda.synchronize()
    L, rge, rgd = oc.loss_eq8_and_grad(we, wd, A, B, T, W)
    assert abs(float(loss) - L) <= 1e-12 * L
    assert np.allclose(to_np(ge), rge, rtol=1e-10, atol=1e-13 * np.abs(rge).max())
    assert np.allclose(to_np(gd), rgd, rtol=1e-10, atol=1e-13 * np.abs(rgd).max())
    h = 1e-6
    scale = max(np.abs(rge).max(), np.abs(rgd).max())
    for which in ("E", "D"):
        for _ in range(3):
            if which == "E":
                idx = (int(rng.integers(k)), int(rng.integers(n)))
                wp, wm = we.copy(), we.copy()
                wp[idx] += h
                wm[idx] -= h
                fd = (oc.loss_eq8(wp, wd, A, B, T, W) - oc.loss_eq8(wm, wd, A, B, T, W)) / (2 * h)
                got = to_np(ge)[idx]
            else:
                idx = (int(rng.integers(n)), int(rng.integers(k)))
                wp, wm = wd.copy(), wd.copy()
                wp[idx] += h
                wm[idx] -= h
                fd = (oc.loss_eq8(we, wp, A, B, T, W) - oc.loss_eq8(we, wm, A, B, T, W)) / (2 * h)
                got = to_np(gd)[idx]
            assert abs(fd - got) <= 1e-7 * scale


def test_eq8_gather_by_index_equals_explicit_batch_and_is_deterministic(ops):
    n, k, N = 81, 9, 5000
    rng = np.random.default_rng(23)
    we, wd = synth.codec_init(rng, k, n)
    pa, pb = _pairs(n, 20000, 24)
    ia = synth.uniform_indices(3, 0, N, 20000)
    ib = synth.uniform_indices(4, 0, N, 20000)
    T = _t(synth.cmf_matrix(n))
    runs = []
    for gather in (True, True, False):
        g = [torch.empty(k, n, device="cuda"), torch.empty(n, k, device="cuda")]
        if gather:
            loss = ops.codec_step(_t(we), _t(wd), _t(pa), _t(pb), N, idx_a=_t(ia.view(np.int32), np.int32),
                                  idx_b=_t(ib.view(np.int32), np.int32), grad_e=g[0], grad_d=g[1],
                                  objective="eq8", T=T)
        else:
            loss = ops.codec_step(_t(we), _t(wd), _t(pa[ia]), _t(pb[ib]), N, grad_e=g[0], grad_d=g[1],
                                  objective="eq8", T=T)
        runs.append((loss.clone(), *g))
    torch.cuda.synchronize()
    for r in runs[1:]:
        assert all(torch.equal(x, y) for x, y in zip(runs[0], r))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_eq8_adam_steps_match_oracle(ops, dtype):
    n, k, N = 31, 6, 2048
    rng = np.random.default_rng(25)
    we, wd = (x.astype(np.float64) for x in synth.codec_init(rng, k, n))
    A, B = _pairs(n, N, 26)
    T = synth.cmf_matrix(n)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    Wt_E, Wt_D, At, Bt, Tt = (_t(x, npdt) for x in (we, wd, A, B, T))
    st = dict(m_E=torch.zeros_like(Wt_E), v_E=torch.zeros_like(Wt_E), m_D=torch.zeros_like(Wt_D),
              v_D=torch.zeros_like(Wt_D), step=torch.zeros(1, dtype=torch.int64, device="cuda"),
              lr=1e-3)
    opt = oc.Adam([we.shape, wd.shape], lr=1e-3)
    ref = [we.astype(npdt).astype(np.float64), wd.astype(npdt).astype(np.float64)]
    Ar, Br, Tr = (x.astype(npdt) for x in (A, B, T))
    weak = [np.full(we.shape, np.inf), np.full(wd.shape, np.inf)]
    for _ in range(10):
        ops.codec_step(Wt_E, Wt_D, At, Bt, N, adam=st, objective="eq8", T=Tt)
        _, ge, gd = oc.loss_eq8_and_grad(ref[0], ref[1], Ar, Br, Tr)
        top = max(np.abs(ge).max(), np.abs(gd).max())
        weak = [np.minimum(weak[0], np.abs(ge) / top), np.minimum(weak[1], np.abs(gd) / top)]
        ref = opt.step(ref, [ge, gd])
    torch.cuda.synchronize()
    assert int(st["step"].item()) == 10
    if dtype == torch.float64:
        assert np.allclose(to_np(Wt_E), ref[0], rtol=1e-10, atol=1e-12)
        assert np.allclose(to_np(Wt_D), ref[1], rtol=1e-10, atol=1e-12)
    else:
        # where |g| sits at the float32 rounding level Adam's sign(g) step is
        # not determined; elsewhere the weights agree to float32 rounding
        for got, want, w in zip((to_np(Wt_E), to_np(Wt_D)), ref, weak):
            firm = w > 1e-4
            assert firm.mean() > 0.95
            assert np.abs(got - want)[firm].max() <= 2e-6
            assert np.abs(got - want).max() <= 2 * 10 * 1e-3


def test_eq8_autograd_gradcheck_fp64(ops):
    from paper_2602_18741_amd.autograd import CodecLossEq8
    rng = np.random.default_rng(27)
    we, wd = (torch.from_numpy(x.astype(np.float64)).cuda().requires_grad_(True)
              for x in synth.codec_init(rng, 6, 31))
    A, B = (_t(x, np.float64) for x in _pairs(31, 300, 28))
    T = _t(synth.cmf_matrix(31), np.float64)
    assert torch.autograd.gradcheck(lambda e, d: CodecLossEq8.apply(e, d, A, B, T, W, 10.0, 1e-8),
                                    (we, wd), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_eq8_autograd_backward_matches_oracle(ops):
    from paper_2602_18741_amd.autograd import codec_loss_eq8
    rng = np.random.default_rng(29)
    we0, wd0 = synth.codec_init(rng, 9, 81)
    A, B = _pairs(81, 4096, 30)
    T = synth.cmf_matrix(81)
    we = _t(we0).requires_grad_(True)
    wd = _t(wd0).requires_grad_(True)
    loss = codec_loss_eq8(we, wd, _t(A), _t(B), _t(T))
    (2.5 * loss).backward()
    L, ge, gd = oc.loss_eq8_and_grad(we0, wd0, A, B, T)
    assert abs(float(loss.detach()) - L) <= 1e-5 * L
    assert _grad_ok(to_np(we.grad), 2.5 * ge) and _grad_ok(to_np(wd.grad), 2.5 * gd)


def test_eq8_degenerate_pairs(ops):
    """Pairs whose product is zero (disjoint supports) and pairs that are
    all zero: the clamped cosine keeps every value finite and equal to the
    oracle's."""
    n, k, N = 31, 6, 64
    rng = np.random.default_rng(31)
    we, wd = (x.astype(np.float64) for x in synth.codec_init(rng, k, n))
    A, B = (x.astype(np.float64) for x in _pairs(n, N, 32))
    A[:8, 16:] = 0.0
    B[:8, :16] = 0.0                      # t = 0 on the first 8 pairs
    A[8:12] = 0.0                          # a = 0: u = 0, S_hat = 0
    T = synth.cmf_matrix(n).astype(np.float64)
    d = np.float64
    ge = torch.empty(k, n, dtype=torch.float64, device="cuda")
    gd = torch.empty(n, k, dtype=torch.float64, device="cuda")
    loss = ops.codec_step(_t(we, d), _t(wd, d), _t(A, d), _t(B, d), N, grad_e=ge, grad_d=gd,
                          objective="eq8", T=_t(T, d))
    torch.cuda.synchronize()
    L, rge, rgd = oc.loss_eq8_and_grad(we, wd, A, B, T)
    assert np.isfinite(float(loss)) and abs(float(loss) - L) <= 1e-12 * L
    assert np.allclose(to_np(ge), rge, rtol=1e-10, atol=1e-13 * np.abs(rge).max())
    assert np.allclose(to_np(gd), rgd, rtol=1e-10, atol=1e-13 * np.abs(rgd).max())


@pytest.mark.parametrize("n,k", [(31, 6), (81, 9)])
@pytest.mark.parametrize("N", [1, 31, 33])
def test_eq8_tiny_batches_fp32(ops, n, k, N):
    """Batches smaller than one wavefront's pairs (the lanes past the batch
    carry zero pairs) on the few-lanes-per-pair kernels."""
    rng = np.random.default_rng(N + n)
    we, wd = synth.codec_init(rng, k, n)
    A, B = _pairs(n, max(N, 2), 50 + N)
    A, B = A[:N], B[:N]
    T = synth.cmf_matrix(n)
    ge = torch.empty(k, n, device="cuda")
    gd = torch.empty(n, k, device="cuda")
    loss = ops.codec_step(_t(we), _t(wd), _t(A), _t(B), N, grad_e=ge, grad_d=gd, objective="eq8",
                          T=_t(T), weights=W)
    torch.cuda.synchronize()
    L, rge, rgd = oc.loss_eq8_and_grad(we, wd, A, B, T, W)
    assert abs(float(loss) - L) <= 1e-5 * L
    assert _grad_ok(to_np(ge), rge) and _grad_ok(to_np(gd), rgd)


@pytest.mark.parametrize("n,k", [(31, 6), (81, 9)])
def test_eq8_degenerate_pairs_fp32(ops, n, k):
    """The degenerate pairs of the float64 test (products that vanish, an
    all-zero spectrum) on the float32 few-lanes-per-pair kernels: finite, and
    equal to the oracle within the float32 bounds."""
    N = 64
    rng = np.random.default_rng(33)
    we, wd = synth.codec_init(rng, k, n)
    A, B = _pairs(n, N, 34)
    h = n // 2
    A[:8, h:] = 0.0
    B[:8, :h] = 0.0                      # t = 0 on the first 8 pairs
    A[8:12] = 0.0                        # a = 0: u = 0, S_hat = 0
    T = synth.cmf_matrix(n)
    ge = torch.empty(k, n, device="cuda")
    gd = torch.empty(n, k, device="cuda")
    loss = ops.codec_step(_t(we), _t(wd), _t(A), _t(B), N, grad_e=ge, grad_d=gd, objective="eq8", T=_t(T))
    torch.cuda.synchronize()
    L, rge, rgd = oc.loss_eq8_and_grad(we, wd, A.astype(np.float32), B.astype(np.float32), T.astype(np.float32))
    assert np.isfinite(float(loss)) and abs(float(loss) - L) <= 1e-5 * L
    assert np.isfinite(to_np(ge)).all() and np.isfinite(to_np(gd)).all()
    assert _grad_ok(to_np(ge), rge) and _grad_ok(to_np(gd), rgd)
