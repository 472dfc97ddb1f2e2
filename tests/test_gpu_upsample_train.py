"""GPU training step of the upsampling network (Sec. 5.2) against the oracle.

Float32 kernels against the FP64 oracle: loss within 1e-5 relative;
gradients normwise within 1e-4, and per element
|g - g_ref| <= 1e-4 max(|g_ref|, 1e-3 |g_ref|_inf) + 3e-5 S.  The first term
is the bar the codec gradients use; the second covers cancellation in the
batch sum: S is the batch mean of the element's per-sample |contribution|,
and the rounding error of a float32 sum scales with the sum of the
magnitudes of its terms, not with the (possibly cancelled) result; 3e-5
allows about 500 float32 operations (2^-24 each) from input to element.

The max-abs term picks a channel per sample, an integer decision taken in
floating point: where the two largest |z - z_gt| of a sample are within the
float32 error of z, either channel is a valid subgradient and the kernel may
take the other one than the oracle's first-largest.  The batches keep such
samples (and plant exact and near ties); the kernel's gradient must match the
oracle's gradient for some choice among the tied channels, which the check
recovers by least squares over the per-sample differences of the choices.
"""

import numpy as np
import pytest
import torch

from oracle import upsample as ou
from tests.gpu_util import to_np

pytestmark = pytest.mark.gpu

H = 128


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_18741_amd import ops as o
    return o


def _net(k, seed):
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(0, 1.0, (H, 3)), b1=rng.normal(0, 0.3, H),
                W2=rng.normal(0, 1 / np.sqrt(H), (H, H)), b2=rng.normal(0, 0.3, H),
                W3=rng.normal(0, 1 / np.sqrt(H), (k, H)), b3=rng.normal(0, 0.3, k))


def _pack(net):
    return np.concatenate([net[x].ravel() for x in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)


def _unpack(v, k):
    out, o = {}, 0
    for name, shape in (("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (k, H)), ("b3", (k,))):
        n = int(np.prod(shape))
        out[name] = v[o:o + n].reshape(shape)
        o += n
    return out


def _blocked(z, k):
    nb = (k + 2) // 3
    out = np.zeros((z.shape[0], 4 * nb), np.float32)
    for c in range(k):
        out[:, 4 * (c // 3) + c % 3] = z[:, c]
    return out


def _data(net32, k, N, seed, ties=None):
    """rgb, target codes and M; the first `ties` samples (default min(8, N // 16))
    get two channels whose |z - z_gt| tie exactly in FP64 before the targets
    are rounded to float32, or differ by 1e-7 or 1e-6 of the larger."""
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0, 1, (N, 3)).astype(np.float32)
    zg = rng.uniform(0, 1, (N, k)).astype(np.float64)
    ties = min(8, N // 16) if ties is None else min(ties, N)
    if k > 1 and ties:
        z = ou.upsample(net32, rgb[:ties])
        for i in range(ties):
            a, b = rng.choice(k, 2, replace=False)
            t = 0.5 + rng.uniform()
            zg[i] = z[i] + rng.uniform(-0.4, 0.4, k) * t
            zg[i, a] = z[i, a] - t
            zg[i, b] = z[i, b] + t * (1.0 + (0.0, 1e-7, -1e-6)[i % 3])
    M = rng.uniform(0.05, 0.5, (3, k)).astype(np.float32)
    return rgb, zg.astype(np.float32), M


ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def _grad_ok(g, ref, scale):
    g, ref, scale = (np.asarray(x, np.float64) for x in (g, ref, scale))
    floor = 1e-3 * np.abs(ref).max()
    elem = (np.abs(g - ref) <= 1e-4 * np.maximum(np.abs(ref), floor) + 3e-5 * scale).all()
    return bool(elem and np.linalg.norm(g - ref) <= 1e-4 * np.linalg.norm(ref))


def _flat(g):
    return np.concatenate([g[x].ravel() for x in ORDER])


def _tie_aware_match(g, net32, rgb, zg, M, white):
    """Whether the kernel gradient g is a subgradient of the batch loss: the
    oracle's gradient with, for each sample whose largest |z - z_gt| is tied
    (within the float32 error of z) between channels, the max-abs term taken
    by any point of the convex hull of the tied channels' terms (the
    subdifferential of a max; a kernel that picks one channel is a vertex of
    it).  The weights are found by bounded least squares over the per-sample
    differences of the choices.  Returns (ok, number of ambiguous samples,
    summed weight moved off the oracle's first-largest channel)."""
    from scipy.optimize import lsq_linear
    N = rgb.shape[0]
    _, g0, sc = ou.upsample_loss_and_grad(net32, rgb, zg, M, white, abs_scale=True)
    ref, scale = _flat(g0), _flat(sc)
    z = ou.upsample(net32, rgb)
    d = np.abs(z - zg.astype(np.float64))
    top = d.max(axis=1)
    eps = 1e-5 * (1.0 + np.abs(z).max(axis=1))          # well above the float32 error of z
    default = np.argmax(d, axis=1)
    cols, alts = [], []
    for i in np.flatnonzero((d >= (top - eps)[:, None]).sum(axis=1) > 1):
        one = lambda c: _flat(ou.upsample_loss_and_grad(  # noqa: E731
            net32, rgb[i:i + 1], zg[i:i + 1], M, white, cstar=[c])[1])
        base = one(default[i])
        for c in np.flatnonzero(d[i] >= top[i] - eps[i]):
            if c != default[i]:
                cols.append((one(c) - base) / N)
                alts.append(i)
    if not cols:
        return _grad_ok(g, ref, scale), 0, 0.0
    A = np.stack(cols, axis=1)
    w = lsq_linear(A, np.asarray(g, np.float64) - ref, bounds=(0.0, 1.0)).x
    per = np.zeros(N)
    np.add.at(per, np.array(alts), w)                    # weight off the default, per sample
    ok = per.max() <= 1.0 + 1e-9 and _grad_ok(g, ref + A @ w, scale)
    return bool(ok), len(set(alts)), float(w.sum())


WHITE = (0.95, 1.0, 1.08)


@pytest.mark.parametrize("k,N", [(6, 4096), (6, 1), (9, 3), (9, 1001), (48, 257), (16, 64)])
def test_loss_and_gradient_match_oracle(ops, k, N):
    p = _pack(_net(k, k + N))
    net32 = _unpack(p, k)
    rgb, zg, M = _data(net32, k, N, 7 + k)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    params = t(p)
    grad = torch.empty_like(params)
    loss = ops.upsample_train_step(params, t(rgb), t(_blocked(zg, k)), t(M), WHITE, k, N, grad=grad)
    torch.cuda.synchronize()
    L = ou.upsample_loss(net32, rgb, zg, M, np.array(WHITE))
    assert abs(float(loss) - L) <= 1e-5 * L
    ok, n_amb, flipped = _tie_aware_match(to_np(grad), net32, rgb, zg, M, np.array(WHITE))
    assert ok, (n_amb, flipped)
    assert n_amb >= min(8, N // 16)


def test_planted_ties_accept_either_channel(ops):
    """A batch where a quarter of the samples tie (exactly, or to 1e-7 and
    1e-6) between two channels of the max-abs term: the kernel's gradient is
    the oracle's for some choice among each tie."""
    k, N = 9, 512
    p = _pack(_net(k, 99))
    net32 = _unpack(p, k)
    rgb, zg, M = _data(net32, k, N, 100, ties=N // 4)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    grad = torch.empty(p.size, device="cuda")
    loss = ops.upsample_train_step(t(p), t(rgb), t(_blocked(zg, k)), t(M), WHITE, k, N, grad=grad)
    torch.cuda.synchronize()
    L = ou.upsample_loss(net32, rgb, zg, M, np.array(WHITE))
    assert abs(float(loss) - L) <= 1e-5 * L
    ok, n_amb, flipped = _tie_aware_match(to_np(grad), net32, rgb, zg, M, np.array(WHITE))
    assert ok and n_amb >= N // 4, (n_amb, flipped)


def test_gather_by_index_equals_explicit_batch_and_is_deterministic(ops):
    k, N = 6, 3000
    p = _pack(_net(k, 3))
    rgb, zg, M = _data(_unpack(p, k), k, 5000, 4)
    idx = np.random.default_rng(5).integers(0, rgb.shape[0], N).astype(np.int32)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    zb = _blocked(zg, k)
    outs = []
    for gather in (True, True, False):
        grad = torch.empty(p.size, device="cuda")
        if gather:
            loss = ops.upsample_train_step(t(p), t(rgb), t(zb), t(M), WHITE, k, N, idx=t(idx), grad=grad)
        else:
            loss = ops.upsample_train_step(t(p), t(rgb[idx]), t(zb[idx]), t(M), WHITE, k, N, grad=grad)
        outs.append((loss.clone(), grad))
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])


@pytest.mark.parametrize("max_norm", [1e-3, 1e6])
def test_adamw_step_matches_oracle_on_the_kernel_gradient(ops, max_norm):
    """Three fused steps (gradient, clipping, AdamW) against the oracle's
    AdamW fed the gradient the kernel reports for the same parameters; with
    max_norm 1e-3 clipping engages on every step, with 1e6 never."""
    k, N = 9, 2048
    p0 = _pack(_net(k, 11))
    rgb, zg, M = _data(_unpack(p0, k), k, N, 12)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    args = (t(rgb), t(_blocked(zg, k)), t(M), WHITE, k, N)
    params = t(p0)
    opt = dict(m=torch.zeros_like(params), v=torch.zeros_like(params),
               step=torch.zeros(1, dtype=torch.int64, device="cuda"), lr=2e-3, weight_decay=1e-5,
               max_grad_norm=max_norm)
    ref_opt = ou.AdamW([p0.shape], lr=2e-3, weight_decay=1e-5, max_norm=max_norm)
    ref = [p0.astype(np.float64)]
    norms = []
    for _ in range(3):
        g = torch.empty_like(params)
        ops.upsample_train_step(params.clone(), *args, grad=g)
        g = to_np(g).astype(np.float64)
        norms.append(np.linalg.norm(g))
        ops.upsample_train_step(params, *args, opt=opt)
        ref = ref_opt.step(ref, [g])
    torch.cuda.synchronize()
    assert int(opt["step"].item()) == 3
    assert (min(norms) > max_norm) == (max_norm < 1)
    got = to_np(params).astype(np.float64)
    # each step moves a weight by at most about lr; float32 rounding of the
    # parameters and moments stays far below that
    assert np.abs(got - ref[0]).max() <= 1e-6 + 1e-6 * np.abs(ref[0]).max()


def test_short_fit_reduces_the_loss(ops):
    from paper_2602_18741_amd.upsample_fit import UpsampleFit
    k = 6
    rng = np.random.default_rng(13)
    rgb = rng.uniform(0, 1, (1 << 14, 3)).astype(np.float32)
    A = rng.uniform(0, 1, (k, 3))
    zg = (rgb @ A.T + 0.1 * np.sin(3 * rgb[:, :1])).astype(np.float32)    # a smooth target
    M = rng.uniform(0.05, 0.5, (3, k)).astype(np.float32)
    fit = UpsampleFit(torch.from_numpy(rgb).cuda(), torch.from_numpy(_blocked(zg, k)).cuda(),
                      torch.from_numpy(M).cuda(), WHITE, k, batch=1024, seed=1)
    first = float(fit.run(1))
    fit.capture()
    last = float(fit.run(300))
    assert last < 0.3 * first


def test_multi_step_graph_replay_equals_eager_steps(ops):
    """Four steps per graph replay (each drawing its batch from the device
    counter at replay time), then single steps: parameters and optimizer
    state equal eager steps bit for bit."""
    from paper_2602_18741_amd.upsample_fit import UpsampleFit
    k = 6
    rng = np.random.default_rng(17)
    rgb = rng.uniform(0, 1, (1 << 13, 3)).astype(np.float32)
    zg = (rgb @ rng.uniform(0, 1, (k, 3)).T).astype(np.float32)
    M = rng.uniform(0.05, 0.5, (3, k)).astype(np.float32)

    def make():
        return UpsampleFit(torch.from_numpy(rgb).cuda(), torch.from_numpy(_blocked(zg, k)).cuda(),
                           torch.from_numpy(M).cuda(), WHITE, k, batch=512, seed=2)
    eager = make()
    eager.run(15)
    graphed = make()
    graphed.run(1)
    graphed.capture(4)
    graphed.run(14)          # three replays, then two single steps
    torch.cuda.synchronize()
    assert graphed.steps_done == eager.steps_done == 15
    for name in ("m", "v", "step"):
        assert torch.equal(eager.opt[name], graphed.opt[name])
    assert torch.equal(eager.params, graphed.params) and torch.equal(eager.loss, graphed.loss)


def test_drawn_rows_equal_generated_indices(ops):
    """Rows drawn inside the training step are the rows hc_gen_indices writes
    for the same seed and counters: loss, gradient-driven parameters and
    optimizer state equal bit for bit over three AdamW steps whose draws take
    their counter base from the step counter."""
    k, N, rows = 6, 1000, 5000
    rng = np.random.default_rng(23)
    rgb = torch.from_numpy(rng.uniform(0, 1, (rows, 3)).astype(np.float32)).cuda()
    z = torch.from_numpy(_blocked(rng.uniform(0, 1, (rows, k)).astype(np.float32), k)).cuda()
    M = torch.from_numpy(rng.uniform(0.05, 0.5, (3, k)).astype(np.float32)).cuda()
    from paper_2602_18741_amd.upsample_fit import default_init
    runs = []
    for use_draw in (False, True):
        params = torch.from_numpy(default_init(k, 3)).cuda()
        opt = dict(m=torch.zeros_like(params), v=torch.zeros_like(params),
                   step=torch.full((1,), 4, dtype=torch.int64, device="cuda"), lr=2e-3)
        out = []
        for _ in range(3):
            if use_draw:
                loss = ops.upsample_train_step(params, rgb, z, M, WHITE, k, N, opt=opt,
                                               draw=dict(seed=11, ctr0=2, step=opt["step"]))
            else:
                idx = ops.gen_indices(11, N, rows, ctr0=2, step=opt["step"])
                loss = ops.upsample_train_step(params, rgb, z, M, WHITE, k, N, idx=idx, opt=opt)
            out.append(loss.clone())
        torch.cuda.synchronize()
        assert int(opt["step"].item()) == 7
        runs.append(out + [params, opt["m"], opt["v"]])
    assert all(torch.equal(x, y) for x, y in zip(*runs))


def test_plateau_schedule_with_graph_recapture_equals_eager(ops):
    """run_epochs with the plateau rule: every round lowers the rate
    (threshold 1: no loss counts as better, the first one included), the graph
    is recorded again
    after each change, and the result equals the same schedule run eagerly,
    bit for bit."""
    from paper_2602_18741_amd.upsample_fit import PlateauLR, UpsampleFit
    k = 6
    rng = np.random.default_rng(29)
    rgb = rng.uniform(0, 1, (1 << 12, 3)).astype(np.float32)
    zg = (rgb @ rng.uniform(0, 1, (k, 3)).T).astype(np.float32)
    M = rng.uniform(0.05, 0.5, (3, k)).astype(np.float32)

    def make():
        return UpsampleFit(torch.from_numpy(rgb).cuda(), torch.from_numpy(_blocked(zg, k)).cuda(),
                           torch.from_numpy(M).cuda(), WHITE, k, batch=256, seed=5)
    eager = make()
    l_e = eager.run_epochs(5, 3, PlateauLR(2e-3, patience=0, threshold=1.0))
    graphed = make()
    graphed.run(1)
    graphed.capture(3)
    graphed.opt["step"].zero_()
    graphed.params.copy_(make().params)
    for name in ("m", "v"):
        graphed.opt[name].zero_()
    l_g = graphed.run_epochs(5, 3, PlateauLR(2e-3, patience=0, threshold=1.0))
    torch.cuda.synchronize()
    assert eager.opt["lr"] == graphed.opt["lr"] == 2e-3 * 0.5 ** 5
    assert l_e == l_g
    assert torch.equal(eager.params, graphed.params)
    assert all(torch.equal(eager.opt[x], graphed.opt[x]) for x in ("m", "v", "step"))


def test_drawn_rows_without_a_counter(ops):
    """A training-step draw with no counter pointer uses the base ctr0 alone."""
    from paper_2602_18741_amd.upsample_fit import default_init
    k, N, rows = 9, 700, 3000
    rng = np.random.default_rng(31)
    rgb = torch.from_numpy(rng.uniform(0, 1, (rows, 3)).astype(np.float32)).cuda()
    z = torch.from_numpy(_blocked(rng.uniform(0, 1, (rows, k)).astype(np.float32), k)).cuda()
    M = torch.from_numpy(rng.uniform(0.05, 0.5, (3, k)).astype(np.float32)).cuda()
    params = torch.from_numpy(default_init(k, 4)).cuda()
    g1 = torch.empty_like(params)
    g2 = torch.empty_like(params)
    l1 = ops.upsample_train_step(params, rgb, z, M, WHITE, k, N, grad=g1, draw=dict(seed=9, ctr0=77))
    idx = ops.gen_indices(9, N, rows, ctr0=77)
    l2 = ops.upsample_train_step(params, rgb, z, M, WHITE, k, N, grad=g2, idx=idx)
    torch.cuda.synchronize()
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
