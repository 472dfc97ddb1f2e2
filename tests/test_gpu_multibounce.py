"""GPU multi-bounce chains (Eq. 10) against the oracle's recurrence.

XYZ bar as for frames: |x - x_ref| <= 2e-5 |x_ref| + 1e-7 per component.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import multibounce as omb
from tests.conftest import xyz_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd import multibounce
    return multibounce


def _inputs(n, k, C, bounces, seed):
    refl, lights = synth.workloads.bounce_chains(n, C, bounces)
    E, D = synth.codec_uniform(np.random.default_rng(seed), k, n)
    return refl, lights, E, D, synth.cmf_matrix(n)


@pytest.mark.parametrize("n,k,C", [(31, 6, 4096), (81, 9, 1027), (31, 31, 300), (31, 9, 1)])
def test_chains_match_oracle(mb, n, k, C):
    from paper_2602_18741_amd import ops
    bounces = 3
    refl, lights, E, D, T = _inputs(n, k, C, bounces, 7)
    dev = "cuda"
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    x0, xs, xl = mb.chain_xyz(t(E), t(D), t(T), ops.padded(t(refl)), ops.padded(t(lights)), k, n,
                              bounces)
    torch.cuda.synchronize()
    r0, rs, rl = omb.chain_xyz(refl.reshape(C, bounces, n), lights, E, D, T)
    assert xyz_close(x0.cpu().numpy(), r0) <= 1.0
    assert xyz_close(xs.cpu().numpy(), rs) <= 1.0
    assert xyz_close(xl.cpu().numpy(), rl) <= 1.0


def test_cie94_report_agrees_with_oracle_chains(mb):
    """The report on the GPU chains equals the report on the oracle's to
    well within the size of the colour errors it measures."""
    from paper_2602_18741_amd import ops
    n, k, C, bounces = 31, 6, 2048, 3
    refl, lights, _, _, T = _inputs(n, k, C, bounces, 8)
    rng = np.random.default_rng(9)
    # a codec close to the identity on 6 broad bands, so the errors are moderate
    E = np.zeros((k, n), np.float32)
    for j in range(k):
        E[j, j * 5:(j + 1) * 5 + 1] = 1.0 / 6
    D = np.ascontiguousarray(E.T * 6 * rng.uniform(0.9, 1.1, (n, k))).astype(np.float32)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    got = mb.cie94_report(*mb.chain_xyz(t(E), t(D), t(T), ops.padded(t(refl)), ops.padded(t(lights)),
                                        k, n, bounces))
    want = mb.cie94_report(*omb.chain_xyz(refl.reshape(C, bounces, n), lights, E, D, T))
    assert [g["bounce"] for g in got] == [1, 2, 3]
    for g, w in zip(got, want):
        assert g["chains"] == w["chains"] > 0
        assert abs(g["mean"] - w["mean"]) <= 1e-3 * max(1.0, w["mean"])
        assert abs(g["p95"] - w["p95"]) <= 1e-2 * max(1.0, w["p95"])
