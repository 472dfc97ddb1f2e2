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

The full objective of Eq. 8 (``eq8_terms``, ``loss_eq8``,
``loss_eq8_and_grad``) weights four terms, each an MSE (mean over the
elements of a pair, then over the batch):

    S_hat = D (E a (.)_B E b),  t = a * b
    L_e2e  = mean_i MSE_i(S_hat, t) (2 - cos_i(S_hat, t))
    L_rec  = MSE(D E a, a) + MSE(D E b, b)
    L_code = MSE(E a (.)_B E b, E t)
    L_col  = MSE(T S_hat, T t)
    L = l_e2e L_e2e + l_rec L_rec + l_code L_code + l_col L_col

The cosine factor is taken per pair (then averaged with the MSE it scales),
with each norm clamped below at eps: cos = x.y / (max(|x|, eps) max(|y|, eps)).
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


# ---------------------------------------------------------------- Eq. 8

EQ8_WEIGHTS = (0.5, 0.75, 1.0, 0.5)   # l_e2e, l_rec, l_code, l_col (Sec. 4.5)


def eq8_terms(E, D, T, A, B, eps: float = 1e-8):
    """The four per-batch terms (L_e2e, L_rec, L_code, L_col) of Eq. 8 for a
    codec given as the matrices E (k x n) and D (n x k) themselves; T is the
    3 x n colour-matching matrix; rows of A and B are the pairs (a_i, b_i)."""
    E, D, T, A, B = _f64(E), _f64(D), _f64(T), _f64(A), _f64(B)
    n, k = D.shape
    U, V = A @ E.T, B @ E.T
    H = U * V                                      # blockwise product (Eq. 6)
    Tg = A * B                                     # spectral product
    S = H @ D.T                                    # decoded product S_hat
    mse = ((S - Tg) ** 2).mean(axis=1)
    ns = np.maximum(np.sqrt((S * S).sum(axis=1)), eps)
    nt = np.maximum(np.sqrt((Tg * Tg).sum(axis=1)), eps)
    cos = (S * Tg).sum(axis=1) / (ns * nt)
    e2e = (mse * (2.0 - cos)).mean()
    rec = ((U @ D.T - A) ** 2).mean() + ((V @ D.T - B) ** 2).mean()
    code = ((H - Tg @ E.T) ** 2).mean()
    col = ((S @ T.T - Tg @ T.T) ** 2).mean()
    return e2e, rec, code, col


def loss_eq8(Wt_E, Wt_D, A, B, T, weights=EQ8_WEIGHTS, beta: float = 10.0,
             eps: float = 1e-8) -> float:
    """Eq. 8 on softplus weights (Eq. 5)."""
    terms = eq8_terms(softplus(Wt_E, beta), softplus(Wt_D, beta), T, A, B, eps)
    return float(sum(w * t for w, t in zip(weights, terms)))


def loss_eq8_and_grad(Wt_E, Wt_D, A, B, T, weights=EQ8_WEIGHTS, beta: float = 10.0,
                      eps: float = 1e-8):
    """Eq. 8 and its gradient with respect to (Wt_E, Wt_D).

    Derivation, per pair with r_h = S_hat - t, M = |r_h|^2 / n,
    c = cos(S_hat, t), and l_* the weights:
      dcos/dS_hat = t / (|S_hat| m_t) - c S_hat / |S_hat|^2   (|S_hat| > eps)
                  = t / (eps m_t)                          (otherwise), m_t = max(|t|, eps)
      g_S  = l_e2e ((2 - c)(2/n) r_h - M dcos/dS_hat) + l_col (2/3) T^T T r_h
      g_h  = D^T g_S + l_code (2/k) (h - E t)
      g_u  = l_rec (2/n) D^T r_a + g_h * v,   g_v = l_rec (2/n) D^T r_b + g_h * u
      dL/dD = l_rec (2/n)(r_a u^T + r_b v^T) + g_S h^T
      dL/dE = g_u a^T + g_v b^T - l_code (2/k)(h - E t) t^T
    averaged over the batch, then times logistic(beta Wt) (Eq. 5).
    Returns (loss, grad_Wt_E k x n, grad_Wt_D n x k)."""
    Wt_E, Wt_D = _f64(Wt_E), _f64(Wt_D)
    E, D = softplus(Wt_E, beta), softplus(Wt_D, beta)
    T, A, B = _f64(T), _f64(A), _f64(B)
    le, lr, lk, lc = weights
    N = A.shape[0]
    n, k = D.shape
    U, V = A @ E.T, B @ E.T
    H = U * V
    Tg = A * B
    S = H @ D.T
    Rh = S - Tg
    Ra, Rb = U @ D.T - A, V @ D.T - B
    Dc = H - Tg @ E.T
    M = (Rh * Rh).sum(axis=1) / n
    sn = np.sqrt((S * S).sum(axis=1))
    ns = np.maximum(sn, eps)
    nt = np.maximum(np.sqrt((Tg * Tg).sum(axis=1)), eps)
    cos = (S * Tg).sum(axis=1) / (ns * nt)
    big = sn > eps
    dcos = Tg / (ns * nt)[:, None]
    dcos -= np.where(big, cos / np.where(big, sn * sn, 1.0), 0.0)[:, None] * S
    Rc = Rh @ T.T                                  # colour residual, N x 3
    L = float(le * (M * (2.0 - cos)).mean() + lr * ((Ra ** 2).sum() + (Rb ** 2).sum()) / (N * n)
              + lk * (Dc ** 2).sum() / (N * k) + lc * (Rc ** 2).sum() / (N * 3))
    gS = le * ((2.0 - cos)[:, None] * (2.0 / n) * Rh - M[:, None] * dcos) + lc * (2.0 / 3.0) * (Rc @ T)
    Gh = gS @ D + lk * (2.0 / k) * Dc
    Gu = lr * (2.0 / n) * (Ra @ D) + Gh * V
    Gv = lr * (2.0 / n) * (Rb @ D) + Gh * U
    gD = (lr * (2.0 / n) * (Ra.T @ U + Rb.T @ V) + gS.T @ H) / N
    gE = (Gu.T @ A + Gv.T @ B - lk * (2.0 / k) * (Dc.T @ Tg)) / N
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
