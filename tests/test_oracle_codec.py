"""Pins of the oracle's codec-fit loss, gradient and Adam (no GPU)."""

import math

import numpy as np
import pytest

import synth
from oracle import codec


def test_softplus_closed_forms():
    """Eq. 5 at special points: softplus(0) = ln 2 / beta; far right it is x;
    far left it vanishes; it is never negative."""
    beta = 10.0
    assert codec.softplus(0.0, beta) == pytest.approx(math.log(2.0) / beta, rel=1e-15)
    assert codec.softplus(5.0, beta) == pytest.approx(5.0, rel=1e-15)
    assert codec.softplus(-5.0, beta) < 1e-21
    x = np.linspace(-3, 3, 101)
    assert (codec.softplus(x, beta) > 0).all()
    # against the defining formula where it does not overflow
    xs = np.linspace(-2, 2, 41)
    assert np.allclose(codec.softplus(xs, beta), np.log1p(np.exp(beta * xs)) / beta, rtol=1e-14)


def test_softplus_slope_is_its_derivative():
    beta = 10.0
    x = np.linspace(-1.5, 1.5, 61)
    h = 1e-6
    fd = (codec.softplus(x + h, beta) - codec.softplus(x - h, beta)) / (2 * h)
    assert np.allclose(codec.softplus_slope(x, beta), fd, rtol=1e-8, atol=1e-12)
    assert codec.softplus_slope(0.0, beta) == 0.5


def _pairs(n, N, seed):
    rng = np.random.default_rng(seed)
    a = synth.reflectances(rng, n, N).astype(np.float64)
    b = synth.illuminant_table(rng, n, N // 2, N - N // 2).astype(np.float64)
    return a, b


def test_loss_closed_form_with_vanishing_codec():
    """With every weight far negative, E and D are ~0, so every residual is
    minus its target: L = mean(|a|^2 + |b|^2 + lam |a*b|^2)."""
    a, b = _pairs(31, 64, 0)
    we, wd = np.full((6, 31), -5.0), np.full((31, 6), -5.0)
    lam = 0.7
    want = ((a * a).sum(1) + (b * b).sum(1) + lam * ((a * b) ** 2).sum(1)).mean()
    assert codec.loss(we, wd, a, b, lam) == pytest.approx(want, rel=1e-12)


def test_loss_closed_form_at_scaled_identity_codec():
    """E = c I, D = d I (n = k = 6): u = c a, so r_a = (cd - 1) a, and
    h = c^2 a*b, so r_h = (c^2 d - 1) a*b.  Hence
    L = mean((cd - 1)^2 (|a|^2 + |b|^2) + lam (c^2 d - 1)^2 |a*b|^2).
    Off-diagonal weights sit at -5, where softplus is ~1e-23."""
    beta, c, d, lam = 10.0, 0.8, 1.7, 1.3
    inv = lambda y: np.log(np.expm1(beta * y)) / beta  # softplus^-1
    we = np.full((6, 6), -5.0)
    wd = np.full((6, 6), -5.0)
    np.fill_diagonal(we, inv(c))
    np.fill_diagonal(wd, inv(d))
    rng = np.random.default_rng(2)
    a, b = rng.uniform(size=(2, 40, 6))
    want = ((c * d - 1) ** 2 * ((a * a).sum(1) + (b * b).sum(1))
            + lam * (c * c * d - 1) ** 2 * ((a * b) ** 2).sum(1)).mean()
    assert codec.loss(we, wd, a, b, lam, beta) == pytest.approx(want, rel=1e-12)
    # the exact identity codec reproduces every product: zero loss
    np.fill_diagonal(we, inv(1.0))
    np.fill_diagonal(wd, inv(1.0))
    assert codec.loss(we, wd, a, b, lam, beta) < 1e-25


@pytest.mark.parametrize("seed", range(16))
def test_gradient_matches_central_differences(seed):
    """Analytic gradient vs FP64 central differences at 16 random N(0, 0.1)
    parameter points; each checked element within 1e-7 of the gradient's
    largest magnitude."""
    rng = np.random.default_rng(100 + seed)
    n, k = 31, 6
    we, wd = synth.codec_init(rng, k, n)
    we, wd = we.astype(np.float64), wd.astype(np.float64)
    a, b = _pairs(n, 256, seed)
    L, ge, gd = codec.loss_and_grad(we, wd, a, b, 1.0)
    assert L == pytest.approx(codec.loss(we, wd, a, b, 1.0), rel=1e-14)
    h = 1e-6
    scale = max(np.abs(ge).max(), np.abs(gd).max())
    for which, g, w in (("E", ge, we), ("D", gd, wd)):
        for idx in [tuple(rng.integers(0, s) for s in w.shape) for _ in range(12)]:
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            if which == "E":
                fd = (codec.loss(wp, wd, a, b) - codec.loss(wm, wd, a, b)) / (2 * h)
            else:
                fd = (codec.loss(we, wp, a, b) - codec.loss(we, wm, a, b)) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-7 * scale, (which, idx, fd, g[idx])


def test_gradient_of_lambda_zero_is_linear_autoencoder():
    """lam = 0 leaves the reconstruction terms only; their gradient is the
    linear autoencoder one, dL/dD = (2/N) sum r x^T (E x)^T over x in {a, b}."""
    rng = np.random.default_rng(7)
    we, wd = synth.codec_init(rng, 6, 31)
    a, b = _pairs(31, 128, 7)
    _, ge, gd = codec.loss_and_grad(we, wd, a, b, 0.0)
    E, D = codec.softplus(we), codec.softplus(wd)
    gD = np.zeros((31, 6))
    gE = np.zeros((6, 31))
    for x in np.concatenate([a, b]):
        u = E @ x
        r = D @ u - x
        gD += 2 * np.outer(r, u)
        gE += 2 * np.outer(D.T @ r, x)
    gD /= a.shape[0]
    gE /= a.shape[0]
    assert np.allclose(gd, gD * codec.softplus_slope(wd), rtol=1e-10, atol=1e-14)
    assert np.allclose(ge, gE * codec.softplus_slope(we), rtol=1e-10, atol=1e-14)


def test_product_term_is_positive_when_k_below_n():
    """Sec. 3.1: no k < n code preserves the Hadamard product for all
    spectra, so the product residual of a generic codec is positive."""
    rng = np.random.default_rng(3)
    we, wd = synth.codec_init(rng, 6, 31)
    a, b = _pairs(31, 64, 3)
    assert codec.loss(we, wd, a, b, 1.0) > codec.loss(we, wd, a, b, 0.0) > 0


def test_adam_matches_torch():
    """The oracle's Adam against torch.optim.Adam (an independent library
    implementation) over 50 steps of a fixed gradient sequence."""
    import torch
    rng = np.random.default_rng(9)
    w0 = [rng.normal(size=(6, 31)), rng.normal(size=(31, 6))]
    grads = [[rng.normal(size=s.shape) * 10 ** rng.uniform(-3, 1) for s in w0] for _ in range(50)]
    opt = codec.Adam([w.shape for w in w0], lr=1e-3)
    ws = [w.copy() for w in w0]
    tp = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in w0]
    topt = torch.optim.Adam(tp, lr=1e-3)
    for g in grads:
        ws = opt.step(ws, g)
        for p, gi in zip(tp, g):
            p.grad = torch.tensor(gi, dtype=torch.float64)
        topt.step()
    for w, p in zip(ws, tp):
        assert np.allclose(w, p.detach().numpy(), rtol=1e-12, atol=1e-14)
