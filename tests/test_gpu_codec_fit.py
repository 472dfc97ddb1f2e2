"""The GPU codec-fit loop: graph replay, checkpoint/resume, convergence."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fitcls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd.codec_fit import CodecFit
    return CodecFit


@pytest.fixture(scope="module")
def pools():
    pa, pb = synth.workloads.codec_pools(31, 1 << 14)
    return torch.from_numpy(pa).cuda(), torch.from_numpy(pb).cuda()


def _fit(fitcls, pools, **kw):
    we0, wd0 = synth.codec_init(np.random.default_rng(5), 6, 31)
    return fitcls(we0, wd0, pools[0], pools[1], batch=4096, seed=3, **kw)


def _same(a, b):
    return torch.equal(a.Wt_E, b.Wt_E) and torch.equal(a.Wt_D, b.Wt_D) and \
        all(torch.equal(a.adam[x], b.adam[x]) for x in ("m_E", "v_E", "m_D", "v_D", "step"))


@pytest.mark.parametrize("per_graph", [1, 4])
def test_graph_replay_equals_eager_steps(fitcls, pools, per_graph):
    """Graphs of one step and of four steps (each step drawing its pairs from
    the device counter at replay time) equal eager steps bit for bit."""
    eager = _fit(fitcls, pools)
    eager.run(16)
    graphed = _fit(fitcls, pools)
    graphed.run(1)
    graphed.capture(per_graph)
    for _ in range(3):           # replays separated by host work and syncs
        graphed.run(per_graph)
        torch.cuda.synchronize()
        _ = float(graphed.loss)
    graphed.run(15 - 3 * per_graph)   # whole replays, then single steps
    torch.cuda.synchronize()
    assert graphed.steps_done == eager.steps_done == 16
    assert _same(eager, graphed) and torch.equal(eager.loss, graphed.loss)


def test_checkpoint_resume_is_bitwise(fitcls, pools, tmp_path):
    full = _fit(fitcls, pools)
    full.run(20)
    half = _fit(fitcls, pools)
    half.run(10)
    path = str(tmp_path / "codec.npz")
    half.save(path)
    resumed = _fit(fitcls, pools)
    resumed.load(path)
    resumed.run(10)
    torch.cuda.synchronize()
    assert _same(full, resumed)


def test_fit_reduces_the_loss(fitcls, pools):
    f = _fit(fitcls, pools, lr=3e-3)
    first = float(f.run(1))
    last = float(f.run(300))
    assert last < 0.5 * first
    E, D = f.weights()
    assert (E >= 0).all() and (D >= 0).all()


def test_eq8_fit_graph_replay_and_descent(fitcls, pools):
    """The Eq. 8 objective through the same loop: graph replays equal eager
    steps bitwise, and 300 steps reduce the loss."""
    T = synth.cmf_matrix(31)
    eager = _fit(fitcls, pools, objective="eq8", T=T)
    eager.run(6)
    graphed = _fit(fitcls, pools, objective="eq8", T=T)
    graphed.run(1)
    graphed.capture()
    graphed.run(5)
    torch.cuda.synchronize()
    assert _same(eager, graphed) and torch.equal(eager.loss, graphed.loss)
    f = _fit(fitcls, pools, objective="eq8", T=T, lr=3e-3)
    first = float(f.run(1))
    last = float(f.run(300))
    assert last < 0.5 * first
