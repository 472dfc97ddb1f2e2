"""hc_codec_step_static (no workspace; the library's static device scratch)
against hc_codec_step with a caller workspace: loss, gradients and Adam state
bit for bit, on two calls in a row, the second with a smaller batch, so that
what the first call left in the shared scratch cannot leak into the second.
Covers the float32 few-lanes-per-pair kernel (n = 31), the matrix-core tile
kernel (n = 81), the generic tiled kernels, float64, both objectives and the
device pair draw."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _setup(k, n, rows, dtype, seed):
    rng = np.random.default_rng(seed)
    we, wd = synth.codec_init(rng, k, n)
    a = synth.reflectances(rng, n, rows)
    b = synth.illuminant_table(rng, n, rows // 2, rows - rows // 2, 5.0, 15.0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)  # noqa: E731
    return t(we), t(wd), t(a), t(b), t(synth.cmf_matrix(n))


def _step(ops, we, wd, A, B, T, N, objective, static, adam, draw):
    k, n = we.shape
    ge, gd = torch.full_like(we, float("nan")), torch.full_like(wd, float("nan"))
    loss = torch.full((), float("nan"), dtype=we.dtype, device="cuda")
    ws = None
    if not static:
        ws = ops.CodecWorkspace(k, n, N, "cuda")
        ws.buf.fill_(0xFF)                       # NaN bytes: nothing may be read unwritten
    st = None
    if adam:
        st = dict(m_E=torch.zeros_like(we), v_E=torch.zeros_like(we), m_D=torch.zeros_like(wd),
                  v_D=torch.zeros_like(wd), step=torch.full((1,), 3, dtype=torch.int64, device="cuda"),
                  lr=1e-3)
    we, wd = we.clone(), wd.clone()
    dr = dict(seed_a=5, seed_b=6, ctr0=11, step=None if st is None else st["step"]) if draw else None
    ops.codec_step(we, wd, A, B, N, loss=loss, grad_e=ge, grad_d=gd, adam=st, workspace=ws,
                   objective=objective, T=T if objective == "eq8" else None, draw=dr,
                   static_scratch=static)
    out = [loss, ge, gd, we, wd]
    if st is not None:
        out += [st[x] for x in ("m_E", "v_E", "m_D", "v_D", "step")]
    return out


@pytest.mark.parametrize("k,n,dtype,objective,adam,draw", [
    (6, 31, torch.float32, "eq8", True, True),
    (9, 81, torch.float32, "l2", False, False),
    (9, 81, torch.float32, "eq8", True, True),
    (9, 31, torch.float32, "eq8", False, True),
    (5, 40, torch.float32, "l2", True, False),
    (6, 31, torch.float64, "eq8", False, False),
])
def test_static_scratch_equals_the_workspace_call(gpu, k, n, dtype, objective, adam, draw):
    from paper_2602_18741_amd import ops
    we, wd, A, B, T = _setup(k, n, 70_000, dtype, seed=k * n)
    for N in (65536, 3001):                     # the second call smaller than the first
        got = _step(ops, we, wd, A, B, T, N, objective, True, adam, draw)
        ref = _step(ops, we, wd, A, B, T, N, objective, False, adam, draw)
        torch.cuda.synchronize()
        assert torch.isfinite(got[0]).item()
        for g, r in zip(got, ref):
            assert torch.equal(g, r), (N, k, n)
