"""Oracle of the codec fit: softplus weights, loss, analytic gradient, Adam (FP64).

Parameters are the unconstrained matrices Wt_E (k x n) and Wt_D (n x k); the
codec uses E = softplus_beta(Wt_E) and D = softplus_beta(Wt_D) (Eq. 5), so
both are non-negative (Sec. 4.1).

Loss on a batch of N pairs (a_i, b_i) of spectra (rows of A and B):

    u = E a,  v = E b,  h = u (.)_B v              (Eq. 4, Eq. 6)
    r_a = D u - a,  r_b = D v - b,  r_h = D h - a * b
    L = (1/N) sum_i ( |r_a|^2 + |r_b|^2 + lam |r_h|^2 )

The first two terms are the reconstruction loss L_rec of Sec. 4.3, the third
the squared-error part of the end-to-end loss L_e2e (decode of the blockwise
product against the spectral product).  Squared norms are summed over the n
samples and averaged over the batch.
"""

from __future__ import annotations

import numpy as np


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def softplus(x, beta: float = 10.0):
    """(1/beta) log(1 + exp(beta x)) (Eq. 5), evaluated without overflow as
    max(x, 0) + log1p(exp(-beta |x|)) / beta."""
    x = _f64(x)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-beta * np.abs(x))) / beta


def softplus_slope(x, beta: float = 10.0):
    """d softplus_beta / dx = logistic(beta x) = 1 / (1 + exp(-beta x))."""
    x = _f64(x)
    e = np.exp(-beta * np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def _forward(E, D, A, B):
    U = A @ E.T
    V = B @ E.T
    H = U * V
    Ra = U @ D.T - A
    Rb = V @ D.T - B
    Rh = H @ D.T - A * B
    return U, V, H, Ra, Rb, Rh


def loss(Wt_E, Wt_D, A, B, lam: float = 1.0, beta: float = 10.0) -> float:
    E, D = softplus(Wt_E, beta), softplus(Wt_D, beta)
    A, B = _f64(A), _f64(B)
    _, _, _, Ra, Rb, Rh = _forward(E, D, A, B)
    return float(((Ra * Ra).sum() + (Rb * Rb).sum() + lam * (Rh * Rh).sum()) / A.shape[0])


def loss_and_grad(Wt_E, Wt_D, A, B, lam: float = 1.0, beta: float = 10.0):
    """Loss and its gradient with respect to (Wt_E, Wt_D).

    Derivation (chain rule on the definitions above, per pair, then / N):
      dL/dD = 2 (r_a u^T + r_b v^T + lam r_h h^T)
      g_h   = lam D^T r_h
      dL/du = 2 (D^T r_a + g_h * v),  dL/dv = 2 (D^T r_b + g_h * u)
      dL/dE = dL/du a^T + dL/dv b^T
      dL/dWt = dL/dW * logistic(beta Wt)        (derivative of Eq. 5)
    Returns (loss, grad_Wt_E k x n, grad_Wt_D n x k).
    """
    Wt_E, Wt_D = _f64(Wt_E), _f64(Wt_D)
    E, D = softplus(Wt_E, beta), softplus(Wt_D, beta)
    A, B = _f64(A), _f64(B)
    N = A.shape[0]
    U, V, H, Ra, Rb, Rh = _forward(E, D, A, B)
    L = float(((Ra * Ra).sum() + (Rb * Rb).sum() + lam * (Rh * Rh).sum()) / N)
    gD = (2.0 / N) * (Ra.T @ U + Rb.T @ V + lam * (Rh.T @ H))
    Gh = lam * (Rh @ D)
    Gu = Ra @ D + Gh * V
    Gv = Rb @ D + Gh * U
    gE = (2.0 / N) * (Gu.T @ A + Gv.T @ B)
    return L, gE * softplus_slope(Wt_E, beta), gD * softplus_slope(Wt_D, beta)


class Adam:
    """Adam with bias correction (Kingma and Ba, ICLR 2015), as used for
    the codec (Sec. 4.5: Adam, lr 1e-3).  State is float64."""

    def __init__(self, shapes, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros(s) for s in shapes]
        self.v = [np.zeros(s) for s in shapes]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        for i, (w, g) in enumerate(zip(params, grads)):
            g = _f64(g)
            self.m[i] = self.b1 * self.m[i] + (1.0 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1.0 - self.b2) * g * g
            m_hat = self.m[i] / (1.0 - self.b1 ** self.t)
            v_hat = self.v[i] / (1.0 - self.b2 ** self.t)
            out.append(_f64(w) - self.lr * m_hat / (np.sqrt(v_hat) + self.eps))
        return out
