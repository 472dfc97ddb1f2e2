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
