"""Oracle of the latent upsampling network (Sec. 5), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network maps a linear RGB colour to a k-channel latent code with three
fully connected layers, hidden width 128 and SiLU activations between them
(Sec. 5.1):

    h1 = silu(W1 c + b1),  h2 = silu(W2 h1 + b2),  z = W3 h2 + b3

with silu(x) = x * logistic(x) = x / (1 + exp(-x)).  The output layer is
linear (the paper names activations only between the layers).
"""

from __future__ import annotations

import numpy as np


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def silu(x):
    """x / (1 + exp(-x)), evaluated without overflow for large |x|."""
    x = _f64(x)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, x / (1.0 + e), x * e / (1.0 + e))


def mlp_hidden(net: dict, rgb):
    """Hidden activations (h1, h2) for rows of rgb (m x 3)."""
    c = _f64(rgb)
    h1 = silu(c @ _f64(net["W1"]).T + _f64(net["b1"]))
    h2 = silu(h1 @ _f64(net["W2"]).T + _f64(net["b2"]))
    return h1, h2


def upsample(net: dict, rgb):
    """Latent codes z (m x k) of the rows of rgb (m x 3).  net holds W1 (h x 3),
    b1 (h), W2 (h x h), b2 (h), W3 (k x h), b3 (k)."""
    _, h2 = mlp_hidden(net, rgb)
    return h2 @ _f64(net["W3"]).T + _f64(net["b3"])


# ------------------------------------------------------------------ training

_D = 6.0 / 29.0


def lab(xyz, white):
    """CIE 1976 L*a*b* of XYZ rows (any sign) against the white (Xn, Yn, Zn):
    f(t) = t^(1/3) above (6/29)^3, else t / (3 (6/29)^2) + 4/29."""
    t = _f64(xyz) / _f64(white)
    f = np.where(t > _D ** 3, np.cbrt(t), t / (3 * _D * _D) + 4.0 / 29.0)
    return np.stack([116.0 * f[:, 1] - 16.0, 500.0 * (f[:, 0] - f[:, 1]),
                     200.0 * (f[:, 1] - f[:, 2])], axis=1)


def _dlab_dxyz(xyz, white):
    """Jacobian (m x 3 x 3) of lab() with respect to XYZ."""
    t = _f64(xyz) / _f64(white)
    fp = np.where(t > _D ** 3, 1.0 / (3.0 * np.cbrt(np.where(t > _D ** 3, t, 1.0)) ** 2),
                  1.0 / (3 * _D * _D)) / _f64(white)
    J = np.zeros((t.shape[0], 3, 3))
    J[:, 0, 1] = 116.0 * fp[:, 1]
    J[:, 1, 0], J[:, 1, 1] = 500.0 * fp[:, 0], -500.0 * fp[:, 1]
    J[:, 2, 1], J[:, 2, 2] = 200.0 * fp[:, 1], -200.0 * fp[:, 2]
    return J


def upsample_loss(net, rgb, z_gt, M, white, w_max: float = 0.3, w_col: float = 0.05):
    """Training objective of Sec. 5.2 on a batch:
        L = MSE(z, z_gt) + w_max mean_i max_c |z_ic - z_gt,ic|
            + w_col mean_i DeltaE76(Lab(M z_i), Lab(M z_gt,i))
    with z the network output, M = T_cmf D (3 x k, XYZ of a code through the
    frozen decoder) and DeltaE76 the Euclidean distance in CIELAB."""
    z = upsample(net, rgb)
    d = z - _f64(z_gt)
    M = _f64(M)
    de = np.linalg.norm(lab(z @ M.T, white) - lab(_f64(z_gt) @ M.T, white), axis=1)
    return float((d * d).mean() + w_max * np.abs(d).max(axis=1).mean() + w_col * de.mean())


def upsample_loss_and_grad(net, rgb, z_gt, M, white, w_max: float = 0.3, w_col: float = 0.05,
                           abs_scale: bool = False, cstar=None):
    """Loss of upsample_loss and its gradient with respect to every weight.

    Backward, per sample (then / N): with d = z - z_gt,
      dz = (2/k) d + w_max sign(d_c*) e_c*  (c* a channel of largest |d|)
           + w_col M^T J^T (Lab_z - Lab_gt) / DeltaE   (0 where DeltaE = 0),
    J the Jacobian of Lab at M z; then through the layers,
      dW3 = dz h2^T, db3 = dz, dp2 = (W3^T dz) * silu'(p2), dW2 = dp2 h1^T, db2 = dp2,
      dp1 = (W2^T dp2) * silu'(p1), dW1 = dp1 c^T, db1 = dp1,
    silu'(x) = s + x s (1 - s), s = logistic(x).
    The max over channels has one subgradient per channel that attains it;
    c* defaults to the first such channel, and `cstar` (one channel index per
    sample) picks another where several tie.
    Returns (loss, dict of gradients keyed like net); with abs_scale also a
    dict of the batch means of |per-sample contribution| of every element
    (the magnitude that rounding errors of the batch sum scale with)."""
    c = _f64(rgb)
    W1, b1, W2, b2 = (_f64(net[x]) for x in ("W1", "b1", "W2", "b2"))
    W3, b3 = _f64(net["W3"]), _f64(net["b3"])
    M = _f64(M)
    N, k = c.shape[0], W3.shape[0]
    p1 = c @ W1.T + b1
    h1 = silu(p1)
    p2 = h1 @ W2.T + b2
    h2 = silu(p2)
    z = h2 @ W3.T + b3
    d = z - _f64(z_gt)
    ad = np.abs(d)
    if cstar is None:
        cstar = np.argmax(ad, axis=1)
    cstar = np.asarray(cstar, dtype=np.int64)
    lz, lg = lab(z @ M.T, white), lab(_f64(z_gt) @ M.T, white)
    diff = lz - lg
    de = np.linalg.norm(diff, axis=1)
    L = float((d * d).mean() + w_max * ad.max(axis=1).mean() + w_col * de.mean())
    dz = (2.0 / k) * d
    dz[np.arange(N), cstar] += w_max * np.sign(d[np.arange(N), cstar])
    unit = np.where(de[:, None] > 0, diff / np.where(de > 0, de, 1.0)[:, None], 0.0)
    gxyz = np.einsum("nij,ni->nj", _dlab_dxyz(z @ M.T, white), unit)
    dz += w_col * gxyz @ M
    dz /= N

    def dsilu(x):
        s = np.where(x >= 0, 1.0 / (1.0 + np.exp(-np.abs(x))), np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))))
        return s + x * s * (1.0 - s)

    dp2 = (dz @ W3) * dsilu(p2)
    dp1 = (dp2 @ W2) * dsilu(p1)
    grads = dict(W3=dz.T @ h2, b3=dz.sum(0), W2=dp2.T @ h1, b2=dp2.sum(0), W1=dp1.T @ c, b1=dp1.sum(0))
    if not abs_scale:
        return L, grads
    a = np.abs
    scale = dict(W3=a(dz).T @ a(h2), b3=a(dz).sum(0), W2=a(dp2).T @ a(h1), b2=a(dp2).sum(0),
                 W1=a(dp1).T @ a(c), b1=a(dp1).sum(0))
    return L, grads, scale


class AdamW:
    """Decoupled weight decay Adam (Loshchilov and Hutter, ICLR 2019) with
    gradient clipping to a global L2 norm, as the upsampler's training uses
    (Sec. 5.2: AdamW, lr 2e-3, weight decay 1e-5, clipping at norm 1).  Each
    step: g *= min(1, max_norm / (|g| + 1e-6)); w *= 1 - lr wd; then the Adam
    update with bias correction.  State is float64."""

    def __init__(self, sizes, lr=2e-3, weight_decay=1e-5, max_norm=1.0, beta1=0.9, beta2=0.999,
                 eps=1e-8):
        self.lr, self.wd, self.max_norm = lr, weight_decay, max_norm
        self.b1, self.b2, self.eps = beta1, beta2, eps
        self.m = [np.zeros(s) for s in sizes]
        self.v = [np.zeros(s) for s in sizes]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        grads = [_f64(g) for g in grads]
        norm = np.sqrt(sum((g * g).sum() for g in grads))
        scale = min(1.0, self.max_norm / (norm + 1e-6))
        out = []
        for i, (w, g) in enumerate(zip(params, grads)):
            g = g * scale
            w = _f64(w) * (1.0 - self.lr * self.wd)
            self.m[i] = self.b1 * self.m[i] + (1.0 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1.0 - self.b2) * g * g
            m_hat = self.m[i] / (1.0 - self.b1 ** self.t)
            v_hat = self.v[i] / (1.0 - self.b2 ** self.t)
            out.append(w - self.lr * m_hat / (np.sqrt(v_hat) + self.eps))
        return out
