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
