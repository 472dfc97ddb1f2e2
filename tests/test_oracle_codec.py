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


# ------------------------------------------------------------ Eq. 8 objective

def _inv_softplus(y, beta=10.0):
    return np.log(np.expm1(beta * y)) / beta


def test_eq8_closed_form_at_scaled_identity_codec():
    """E = c I, D = d I (k = n = 6): u = c a, h = c^2 t with t = a*b, so
    S_hat = d c^2 t is parallel to t (cos = 1) and every term has a closed form:
      L_e2e = mean (dc^2 - 1)^2 |t|^2 / n,  L_rec = mean (cd - 1)^2 (|a|^2 + |b|^2) / n,
      L_code = mean (c^2 - c)^2 |t|^2 / k,  L_col = mean (dc^2 - 1)^2 |T t|^2 / 3."""
    n, c, d = 6, 0.8, 1.7
    rng = np.random.default_rng(11)
    a, b = rng.uniform(0.05, 1.0, size=(2, 40, n))
    T = rng.uniform(size=(3, n))
    t = a * b
    want = (((d * c * c - 1) ** 2 * (t * t).sum(1) / n).mean(),
            ((c * d - 1) ** 2 * ((a * a).sum(1) + (b * b).sum(1)) / n).mean(),
            ((c * c - c) ** 2 * (t * t).sum(1) / n).mean(),
            ((d * c * c - 1) ** 2 * ((t @ T.T) ** 2).sum(1) / 3).mean())
    got = codec.eq8_terms(c * np.eye(n), d * np.eye(n), T, a, b)
    assert np.allclose(got, want, rtol=1e-13, atol=0)
    # the same through softplus parameters (off-diagonals at -5: softplus ~ 1e-23)
    we, wd = np.full((n, n), -5.0), np.full((n, n), -5.0)
    np.fill_diagonal(we, _inv_softplus(c))
    np.fill_diagonal(wd, _inv_softplus(d))
    w = (0.5, 0.75, 1.0, 0.5)
    assert codec.loss_eq8(we, wd, a, b, T, w) == pytest.approx(np.dot(w, want), rel=1e-12)
    assert codec.loss_eq8_and_grad(we, wd, a, b, T, w)[0] == pytest.approx(np.dot(w, want), rel=1e-12)


def test_eq8_orthogonal_reconstruction_doubles_the_mse():
    """n = k = 2, E = I, D = the swap: t = (1, 0) decodes to (0, 1), which is
    orthogonal to t, so the cosine factor is 2 and L_e2e = 2 MSE = 2; the code
    is exact (L_code = 0); L_rec and L_col follow from the swap."""
    x = 0.3
    a = np.array([[1.0, x]])
    b = np.array([[1.0, 0.0]])
    T = np.array([[0.2, 0.9], [0.5, 0.1], [0.7, 0.4]])
    e2e, rec, code, col = codec.eq8_terms(np.eye(2), np.array([[0.0, 1.0], [1.0, 0.0]]), T, a, b)
    assert e2e == 2.0
    assert rec == pytest.approx((x - 1) ** 2 + 1.0, rel=1e-15)
    assert code == 0.0
    assert col == pytest.approx(((T[:, 1] - T[:, 0]) ** 2).sum() / 3, rel=1e-15)


def test_eq8_code_term_vanishes_for_sample_selecting_encoders():
    """An encoder whose rows each pick one sample commutes with the product,
    E(a*b) = Ea * Eb, so L_code = 0 for any pairs and any decoder."""
    rng = np.random.default_rng(12)
    n, k = 31, 6
    E = np.zeros((k, n))
    E[np.arange(k), rng.choice(n, k, replace=False)] = 1.0
    a, b = _pairs(n, 32, 12)
    assert codec.eq8_terms(E, rng.uniform(size=(n, k)), synth.cmf_matrix(n), a, b)[2] == 0.0


def test_eq8_reconstruction_weight_alone_is_the_scaled_two_term_loss():
    """With weights (0, 1, 0, 0) Eq. 8 is L_rec, the two-term loss at lam = 0
    divided by n (MSE averages over the samples); the gradients scale alike."""
    rng = np.random.default_rng(13)
    n, k = 31, 6
    we, wd = synth.codec_init(rng, k, n)
    a, b = _pairs(n, 64, 13)
    T = synth.cmf_matrix(n)
    L8, ge8, gd8 = codec.loss_eq8_and_grad(we, wd, a, b, T, (0.0, 1.0, 0.0, 0.0))
    L2, ge2, gd2 = codec.loss_and_grad(we, wd, a, b, 0.0)
    assert L8 == pytest.approx(L2 / n, rel=1e-12)
    assert np.allclose(ge8, ge2 / n, rtol=1e-10, atol=0)
    assert np.allclose(gd8, gd2 / n, rtol=1e-10, atol=0)


def test_eq8_terms_match_torch_functional_definitions():
    """Each term against torch's own MSE and cosine-similarity routines
    (float64, CPU), the library meaning of the paper's MSE and cos."""
    import torch
    import torch.nn.functional as F
    rng = np.random.default_rng(14)
    n, k = 81, 9
    we, wd = synth.codec_init(rng, k, n)
    E, D = codec.softplus(we), codec.softplus(wd)
    a, b = _pairs(n, 48, 14)
    T = synth.cmf_matrix(n)
    tE, tD, tT, ta, tb = (torch.tensor(np.asarray(x, np.float64)) for x in (E, D, T, a, b))
    t = ta * tb
    S = ((ta @ tE.T) * (tb @ tE.T)) @ tD.T
    e2e = (F.mse_loss(S, t, reduction="none").mean(1) * (2 - F.cosine_similarity(S, t, dim=1))).mean()
    rec = F.mse_loss(ta @ tE.T @ tD.T, ta) + F.mse_loss(tb @ tE.T @ tD.T, tb)
    code = F.mse_loss((ta @ tE.T) * (tb @ tE.T), t @ tE.T)
    col = F.mse_loss(S @ tT.T, t @ tT.T)
    want = [float(x) for x in (e2e, rec, code, col)]
    assert np.allclose(codec.eq8_terms(E, D, T, a, b), want, rtol=1e-12, atol=0)


def test_eq8_gradient_matches_torch_autograd():
    """The hand-derived Eq. 8 gradient against torch autograd of the same
    objective written with torch's MSE and cosine routines (float64, CPU)."""
    import torch
    import torch.nn.functional as F
    rng = np.random.default_rng(15)
    n, k = 31, 9
    we, wd = synth.codec_init(rng, k, n)
    a, b = _pairs(n, 96, 15)
    T = synth.cmf_matrix(n)
    w = (0.5, 0.75, 1.0, 0.5)
    L, ge, gd = codec.loss_eq8_and_grad(we, wd, a, b, T, w)
    twe = torch.tensor(np.asarray(we, np.float64), requires_grad=True)
    twd = torch.tensor(np.asarray(wd, np.float64), requires_grad=True)
    E, D = F.softplus(twe, beta=10.0, threshold=1e9), F.softplus(twd, beta=10.0, threshold=1e9)
    ta, tb, tT = (torch.tensor(np.asarray(x, np.float64)) for x in (a, b, T))
    t = ta * tb
    u, v = ta @ E.T, tb @ E.T
    S = (u * v) @ D.T
    tl = (w[0] * (F.mse_loss(S, t, reduction="none").mean(1) * (2 - F.cosine_similarity(S, t, dim=1))).mean()
          + w[1] * (F.mse_loss(u @ D.T, ta) + F.mse_loss(v @ D.T, tb))
          + w[2] * F.mse_loss(u * v, t @ E.T) + w[3] * F.mse_loss(S @ tT.T, t @ tT.T))
    tl.backward()
    tl = tl.detach()
    assert L == pytest.approx(tl.item(), rel=1e-12)
    assert np.allclose(ge, twe.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(ge).max())
    assert np.allclose(gd, twd.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(gd).max())


@pytest.mark.parametrize("seed,n,k", [(s, 31, 6) for s in range(4)] + [(s, 81, 9) for s in range(4, 6)])
def test_eq8_gradient_matches_central_differences(seed, n, k):
    """Eq. 8 gradient vs FP64 central differences on a random subset of
    parameters (all of them at n = 31), each within 1e-7 of the largest."""
    rng = np.random.default_rng(200 + seed)
    we, wd = rng.normal(0.0, 0.1, (k, n)), rng.normal(0.0, 0.1, (n, k))
    a, b = _pairs(n, 32, 200 + seed)
    T = synth.cmf_matrix(n)
    _, ge, gd = codec.loss_eq8_and_grad(we, wd, a, b, T)
    scale = max(np.abs(ge).max(), np.abs(gd).max())
    h = 1e-6
    for which, W, g in (("E", we, ge), ("D", wd, gd)):
        idxs = list(np.ndindex(W.shape))
        if n > 31:
            idxs = [idxs[i] for i in rng.choice(len(idxs), 60, replace=False)]
        for idx in idxs:
            wp, wm = W.copy(), W.copy()
            wp[idx] += h
            wm[idx] -= h
            if which == "E":
                fd = (codec.loss_eq8(wp, wd, a, b, T) - codec.loss_eq8(wm, wd, a, b, T)) / (2 * h)
            else:
                fd = (codec.loss_eq8(we, wp, a, b, T) - codec.loss_eq8(we, wm, a, b, T)) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-7 * scale, (which, idx, fd, g[idx])


def test_eq8_cosine_factor_lies_between_one_and_two():
    """Non-negative codecs and spectra give cos in [0, 1], so L_e2e lies
    between the plain MSE and twice it."""
    rng = np.random.default_rng(16)
    we, wd = synth.codec_init(rng, 6, 31)
    E, D = codec.softplus(we), codec.softplus(wd)
    a, b = _pairs(31, 64, 16)
    S = ((a @ E.T) * (b @ E.T)) @ D.T
    mse = ((S - a * b) ** 2).mean()
    e2e = codec.eq8_terms(E, D, synth.cmf_matrix(31), a, b)[0]
    assert mse <= e2e <= 2 * mse
