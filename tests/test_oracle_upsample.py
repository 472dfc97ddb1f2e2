"""Pins of the upsampling-network oracle (Sec. 5) (no GPU)."""

import numpy as np
import pytest

from oracle import upsample as ou


def _net(k, h=128, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(0, scale / np.sqrt(3), (h, 3)), b1=rng.normal(0, 0.1, h),
                W2=rng.normal(0, scale / np.sqrt(h), (h, h)), b2=rng.normal(0, 0.1, h),
                W3=rng.normal(0, scale / np.sqrt(h), (k, h)), b3=rng.normal(0, 0.1, k))


def test_silu_against_scipy_logistic():
    """silu(x) = x * expit(x) with scipy's logistic; silu(0) = 0; far right it
    is x, far left it vanishes; it never overflows."""
    from scipy.special import expit
    x = np.concatenate([np.linspace(-40, 40, 2001), [-1e4, 1e4]])
    assert np.allclose(ou.silu(x), x * expit(x), rtol=1e-14, atol=1e-300)
    assert ou.silu(0.0) == 0.0
    assert ou.silu(50.0) == pytest.approx(50.0, rel=1e-15)
    assert abs(ou.silu(-50.0)) < 1e-19
    assert np.isfinite(ou.silu(np.array([-1e300, 1e300]))).all()


def test_matches_torch_sequential():
    """The network against torch.nn (Linear, SiLU, Linear, SiLU, Linear) in
    float64 on the CPU: the library meaning of the architecture of Sec. 5.1."""
    import torch
    k = 6
    net = _net(k, seed=1)
    seq = torch.nn.Sequential(torch.nn.Linear(3, 128), torch.nn.SiLU(), torch.nn.Linear(128, 128),
                              torch.nn.SiLU(), torch.nn.Linear(128, k)).double()
    with torch.no_grad():
        for lin, w, b in ((seq[0], "W1", "b1"), (seq[2], "W2", "b2"), (seq[4], "W3", "b3")):
            lin.weight.copy_(torch.from_numpy(net[w]))
            lin.bias.copy_(torch.from_numpy(net[b]))
        rgb = np.random.default_rng(2).uniform(size=(500, 3))
        want = seq(torch.from_numpy(rgb)).numpy()
    assert np.allclose(ou.upsample(net, rgb), want, rtol=1e-13, atol=1e-14)


def test_constant_second_layer_gives_constant_code():
    """W2 = 0: h2 = silu(b2) whatever the colour, so z = W3 silu(b2) + b3."""
    net = _net(9, seed=3)
    net["W2"] = np.zeros((128, 128))
    rgb = np.random.default_rng(4).uniform(size=(50, 3))
    want = net["W3"] @ ou.silu(net["b2"]) + net["b3"]
    assert np.allclose(ou.upsample(net, rgb), np.tile(want, (50, 1)), rtol=1e-14, atol=0)


def test_single_path_closed_form():
    """One active unit per layer: W1 row 0 = (1, 2, 3), W2[0, 0] = a, W3[:, 0] = w
    and everything else 0: z = w silu(a silu(r + 2 g + 3 b)) + w0 silu(0) ... with
    zero biases the other units are silu(0) = 0, so z = w silu(a silu(r + 2g + 3b))."""
    k, a = 6, 1.7
    net = {key: np.zeros_like(v) for key, v in _net(k).items()}
    net["W1"][0] = (1.0, 2.0, 3.0)
    net["W2"][0, 0] = a
    w = np.arange(1.0, k + 1.0)
    net["W3"][:, 0] = w
    rgb = np.random.default_rng(5).uniform(size=(20, 3))
    s = rgb @ np.array([1.0, 2.0, 3.0])
    inner = s / (1 + np.exp(-s))
    outer = a * inner / (1 + np.exp(-a * inner))
    assert np.allclose(ou.upsample(net, rgb), outer[:, None] * w[None, :], rtol=1e-14, atol=0)


# ------------------------------------------------------------ training objective

def _batch(k, N, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, 1, (N, 3)), rng.uniform(0, 1, (N, k)), rng.uniform(0.05, 0.5, (3, k)),
            np.array([0.95, 1.0, 1.08]))


def test_lab_closed_forms():
    white = np.array([0.95, 1.0, 1.08])
    assert np.allclose(ou.lab(white[None], white), [[100.0, 0.0, 0.0]], atol=1e-12)
    assert np.allclose(ou.lab(np.zeros((1, 3)), white), [[0.0, 0.0, 0.0]], atol=1e-12)
    t = np.array([0.5, 0.02, 0.001, (6 / 29) ** 3])
    grey = ou.lab(t[:, None] * white[None], white)
    f = np.where(t > (6 / 29) ** 3, np.cbrt(t), t / (3 * (6 / 29) ** 2) + 4 / 29)
    assert np.allclose(grey[:, 0], 116 * f - 16, rtol=1e-13) and np.allclose(grey[:, 1:], 0, atol=1e-12)
    # the two branches meet at (6/29)^3
    e = (6 / 29) ** 3
    lo, hi = ou.lab(np.array([[e, e, e]]) * (1 - 1e-12), np.ones(3)), ou.lab(np.array([[e, e, e]]), np.ones(3))
    assert abs(lo[0, 0] - hi[0, 0]) < 1e-8


def test_mse_only_objective_has_the_linear_output_gradient():
    """w_max = w_col = 0: L = mean (z - z_gt)^2, so dW3 = (2 / (N k)) d^T h2 and
    db3 = (2 / (N k)) sum d, with d = z - z_gt."""
    k, N = 6, 50
    net = _net(k, seed=7)
    rgb, zg, M, white = _batch(k, N, 8)
    L, g = ou.upsample_loss_and_grad(net, rgb, zg, M, white, 0.0, 0.0)
    _, h2 = ou.mlp_hidden(net, rgb)
    d = ou.upsample(net, rgb) - zg
    assert L == pytest.approx((d * d).mean(), rel=1e-14)
    assert np.allclose(g["W3"], 2.0 / (N * k) * d.T @ h2, rtol=1e-12, atol=0)
    assert np.allclose(g["b3"], 2.0 / (N * k) * d.sum(0), rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed", range(3))
def test_training_gradient_matches_central_differences(seed):
    k, N = (6, 9, 16)[seed], 30
    net = _net(k, seed=20 + seed)
    rgb, zg, M, white = _batch(k, N, 30 + seed)
    _, g = ou.upsample_loss_and_grad(net, rgb, zg, M, white)
    scale = max(np.abs(v).max() for v in g.values())
    rng = np.random.default_rng(seed)
    h = 1e-6
    for key in net:
        W = net[key]
        for flat in rng.choice(W.size, min(W.size, 12), replace=False):
            idx = np.unravel_index(flat, W.shape)
            p = dict(net)
            wp, wm = W.copy(), W.copy()
            wp[idx] += h
            wm[idx] -= h
            p[key] = wp
            lp = ou.upsample_loss(p, rgb, zg, M, white)
            p[key] = wm
            lm = ou.upsample_loss(p, rgb, zg, M, white)
            assert abs((lp - lm) / (2 * h) - g[key][idx]) <= 1e-7 * scale, (key, idx)


def test_training_gradient_matches_torch_autograd():
    """The objective written with torch's MSE, amax and norm (float64, CPU),
    differentiated by autograd."""
    import torch
    import torch.nn.functional as F
    k, N = 9, 64
    net = _net(k, seed=40)
    rgb, zg, M, white = _batch(k, N, 41)
    L, g = ou.upsample_loss_and_grad(net, rgb, zg, M, white)
    tn = {key: torch.tensor(v, dtype=torch.float64, requires_grad=True) for key, v in net.items()}
    tc, tz, tM, tw = (torch.tensor(x, dtype=torch.float64) for x in (rgb, zg, M, white))
    h1 = F.silu(tc @ tn["W1"].T + tn["b1"])
    h2 = F.silu(h1 @ tn["W2"].T + tn["b2"])
    z = h2 @ tn["W3"].T + tn["b3"]

    def tlab(xyz):
        t = xyz / tw
        d = 6 / 29
        f = torch.where(t > d ** 3, torch.sign(t) * torch.abs(t).clamp_min(1e-300) ** (1 / 3),
                        t / (3 * d * d) + 4 / 29)
        return torch.stack([116 * f[:, 1] - 16, 500 * (f[:, 0] - f[:, 1]), 200 * (f[:, 1] - f[:, 2])], 1)

    de = torch.linalg.vector_norm(tlab(z @ tM.T) - tlab(tz @ tM.T), dim=1)
    tl = F.mse_loss(z, tz) + 0.3 * (z - tz).abs().amax(dim=1).mean() + 0.05 * de.mean()
    tl.backward()
    assert L == pytest.approx(tl.item(), rel=1e-12)
    for key in net:
        assert np.allclose(g[key], tn[key].grad.numpy(), rtol=1e-9, atol=1e-12), key


def test_adamw_with_clipping_matches_torch():
    """oracle AdamW against torch.optim.AdamW after torch.nn.utils.clip_grad_norm_
    over 30 steps; gradients large enough that clipping engages on some steps."""
    import torch
    rng = np.random.default_rng(50)
    shapes = [(128, 3), (128,), (6, 128)]
    w0 = [rng.normal(size=s) for s in shapes]
    grads = [[rng.normal(size=s) * 10 ** rng.uniform(-3, 0.5) for s in shapes] for _ in range(30)]
    opt = ou.AdamW(shapes, lr=2e-3, weight_decay=1e-5, max_norm=1.0)
    ws = [w.copy() for w in w0]
    tp = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in w0]
    topt = torch.optim.AdamW(tp, lr=2e-3, weight_decay=1e-5)
    clipped = 0
    for g in grads:
        ws = opt.step(ws, g)
        for p, gi in zip(tp, g):
            p.grad = torch.tensor(gi, dtype=torch.float64)
        clipped += float(torch.nn.utils.clip_grad_norm_(tp, 1.0)) > 1.0
        topt.step()
    assert 0 < clipped < 30
    for w, p in zip(ws, tp):
        assert np.allclose(w, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_abs_scale_bounds_the_gradient():
    """The batch mean of |per-sample contribution| bounds |gradient| element
    by element (triangle inequality), with equality for one sample."""
    k = 9
    net = _net(k, seed=60)
    rgb, zg, M, white = _batch(k, 40, 61)
    _, g, sc = ou.upsample_loss_and_grad(net, rgb, zg, M, white, abs_scale=True)
    for key in g:
        assert (np.abs(g[key]) <= sc[key] * (1 + 1e-12) + 1e-300).all()
    _, g1, sc1 = ou.upsample_loss_and_grad(net, rgb[:1], zg[:1], M, white, abs_scale=True)
    for key in g1:
        assert np.allclose(np.abs(g1[key]), sc1[key], rtol=1e-12, atol=0)


def test_tied_max_channels_give_the_one_sided_derivatives():
    """At an exact tie of the two largest |z - z_gt| the max-abs term of
    Sec. 5.2 has a kink: the right-sided derivative along a direction v is the
    larger of the two tied channels' directional derivatives, the left-sided
    one the smaller.  The oracle's gradients with either channel taking the
    term (cstar) must be exactly those two, checked by one-sided differences
    of the loss; with no tie, cstar = argmax reproduces the default."""
    k = 6
    net = _net(k, seed=70)
    rgb, zg, M, white = _batch(k, 1, 71)
    z = ou.upsample(net, rgb)[0]
    a, b, t = 1, 4, 0.9                        # planted tie: d_a = +t, d_b = -t
    zg = z - 0.01 * np.arange(k)               # other |d| well below t
    zg[a], zg[b] = z[a] - t, z[b] + t
    zg = zg[None]
    ga = ou.upsample_loss_and_grad(net, rgb, zg, M, white, cstar=[a])[1]
    gb = ou.upsample_loss_and_grad(net, rgb, zg, M, white, cstar=[b])[1]
    flat = lambda g: np.concatenate([g[x].ravel() for x in sorted(g)])  # noqa: E731
    fa, fb = flat(ga), flat(gb)
    assert np.linalg.norm(fa - fb) > 1e-3 * np.linalg.norm(fa)     # the two subgradients differ
    rng = np.random.default_rng(72)
    keys = sorted(net)
    cuts = np.cumsum([net[x].size for x in keys])[:-1]

    def unflat(f):
        return {x: p.reshape(net[x].shape) for x, p in zip(keys, np.split(f, cuts))}
    # three random directions and the one that separates the two subgradients
    dirs = [rng.normal(size=fa.size) for _ in range(3)] + [(fa - fb) / np.linalg.norm(fa - fb)]
    h = 1e-7
    l0 = ou.upsample_loss(net, rgb, zg, M, white)
    for fv in dirs:
        v = unflat(fv)
        step = lambda s: {x: net[x] + s * v[x] for x in net}  # noqa: E731
        right = (ou.upsample_loss(step(h), rgb, zg, M, white) - l0) / h
        left = (l0 - ou.upsample_loss(step(-h), rgb, zg, M, white)) / h
        hi, lo = max(fa @ fv, fb @ fv), min(fa @ fv, fb @ fv)
        tol = 1e-5 * (abs(hi) + abs(lo) + 1)
        assert abs(right - hi) <= tol and abs(left - lo) <= tol
    assert hi - lo > 100 * tol                  # the last direction resolves the kink
    # no tie: the explicit argmax choice is the default
    rgb2, zg2, M2, _ = _batch(k, 20, 73)
    d = np.abs(ou.upsample(net, rgb2) - zg2)
    g0 = ou.upsample_loss_and_grad(net, rgb2, zg2, M2, white)[1]
    g1 = ou.upsample_loss_and_grad(net, rgb2, zg2, M2, white, cstar=np.argmax(d, axis=1))[1]
    assert all(np.array_equal(g0[x], g1[x]) for x in g0)
