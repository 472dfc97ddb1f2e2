"""GPU training step of the upsampling network (Sec. 5.2) against the oracle.

Float32 kernels against the FP64 oracle: loss within 1e-5 relative;
gradients normwise within 1e-4, and per element
|g - g_ref| <= 1e-4 max(|g_ref|, 1e-3 |g_ref|_inf) + 3e-5 S.  The first term
is the bar the codec gradients use; the second covers cancellation in the
batch sum: S is the batch mean of the element's per-sample |contribution|,
and the rounding error of a float32 sum scales with the sum of the
magnitudes of its terms, not with the (possibly cancelled) result; 3e-5
allows about 500 float32 operations (2^-24 each) from input to element.  The max-abs term picks a channel per sample (an integer
decision taken in floating point); the batches here keep only samples whose
two largest |z - z_gt| differ by more than 1e-3 of the largest, so both
sides take the same decision.
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


def _data(net32, k, N, seed):
    """rgb, target codes and M with well-separated max channels."""
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0, 1, (3 * N, 3)).astype(np.float32)
    zg = rng.uniform(0, 1, (3 * N, k)).astype(np.float32)
    d = np.abs(ou.upsample(net32, rgb) - zg)
    top = np.sort(d, axis=1)
    keep = np.flatnonzero(top[:, -1] - top[:, -2] > 1e-3 * top[:, -1])[:N]
    M = rng.uniform(0.05, 0.5, (3, k)).astype(np.float32)
    return rgb[keep], zg[keep], M


ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def _grad_ok(g, ref, scale):
    g, ref, scale = (np.asarray(x, np.float64) for x in (g, ref, scale))
    floor = 1e-3 * np.abs(ref).max()
    elem = (np.abs(g - ref) <= 1e-4 * np.maximum(np.abs(ref), floor) + 3e-5 * scale).all()
    return bool(elem and np.linalg.norm(g - ref) <= 1e-4 * np.linalg.norm(ref))


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
    L, g, sc = ou.upsample_loss_and_grad(net32, rgb, zg, M, np.array(WHITE), abs_scale=True)
    assert abs(float(loss) - L) <= 1e-5 * L
    ref = np.concatenate([g[x].ravel() for x in ORDER])
    scale = np.concatenate([sc[x].ravel() for x in ORDER])
    assert _grad_ok(to_np(grad), ref, scale)


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
