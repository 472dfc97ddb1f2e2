"""Planted mistakes in the oracle, for tests/test_oracle_mutations.py.

Each entry changes one spot of one oracle module the way a plausible slip
would (a dropped term or factor, a wrong sign, a transposed or permuted
operand, a wrong normaliser, an off-by-one offset).  With HC_ORACLE_MUTANT
naming an entry, tests/conftest.py installs the mutated module before any
test imports the oracle (the other oracle modules are re-imported so that
they use it), and the module's pin tests run against it: every entry must
make at least one of them fail.
"""

from __future__ import annotations

import importlib
import os
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# id: (oracle module, text, replacement, pin test file)
MUTANTS = {
    # shading, encode and decode (Sec. 3, Eq. 4, Eq. 6)
    "shade-light-dropped": ("shade", "acc = lights[light].copy()", "acc = np.ones_like(lights[light])",
                            "test_oracle_shade.py"),
    "shade-weight-dropped": ("shade", "product(acc[live], weight[j][:, None] * table[texel[j]])",
                             "product(acc[live], table[texel[j]])", "test_oracle_shade.py"),
    "shade-vertex-off-by-one": ("shade", "j = first[live] + v\n",
                                "j = np.minimum(first[live] + v + 1, texel.size - 1)\n",
                                "test_oracle_shade.py"),
    "shade-mean-normaliser": ("shade", "sum(axis=1) / spp", "sum(axis=1) / w", "test_oracle_shade.py"),
    "shade-cmf-rows-swapped": ("shade", "return pixel_mean(spec @ _f64(T).T, spp)",
                               "return pixel_mean(spec @ _f64(T)[::-1].T, spp)", "test_oracle_shade.py"),
    "encode-channels-permuted": ("shade", "return _f64(S) @ _f64(E).T", "return _f64(S) @ _f64(E)[::-1].T",
                                 "test_oracle_shade.py"),
    "decode-samples-reversed": ("shade", "s_hat = _f64(Z) @ _f64(D).T", "s_hat = _f64(Z) @ _f64(D)[::-1].T",
                                "test_oracle_shade.py"),
    "blockwise-permuted": ("shade", "za[..., 3 * i:3 * i + 3] * zb[..., 3 * i:3 * i + 3]",
                           "za[..., 3 * i:3 * i + 3] * zb[..., 3 * i:3 * i + 3][..., ::-1]",
                           "test_oracle_shade.py"),
    "latent-sum-not-mean": ("shade", "return pixel_mean(z, spp)", "return pixel_mean(z, spp) * spp",
                            "test_oracle_shade.py"),
    # record format
    "records-length-shift": ("records", "length = (hdr >> 24)", "length = (hdr >> 25)", "test_oracle_shade.py"),
    "records-light-mask": ("records", "light = (hdr & 0xFFFFFF)", "light = (hdr & 0xFFFF)",
                           "test_oracle_shade.py"),
    "records-inclusive-prefix": ("records", "within = np.cumsum(lp, axis=1) - lp",
                                 "within = np.cumsum(lp, axis=1)", "test_oracle_shade.py"),
    "records-weight-cast": ("records", "vtx[:, 1].view(np.float32)", "vtx[:, 1].astype(np.float32)",
                            "test_oracle_shade.py"),
    # codec fit: Eq. 5, the two-term loss and Eq. 8, Adam
    "softplus-scale-dropped": ("codec", "np.log1p(np.exp(-beta * np.abs(x))) / beta",
                               "np.log1p(np.exp(-beta * np.abs(x)))", "test_oracle_codec.py"),
    "slope-branches-swapped": ("codec", "return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))",
                               "return np.where(x >= 0, e / (1.0 + e), 1.0 / (1.0 + e))",
                               "test_oracle_codec.py"),
    "product-target-wrong": ("codec", "Rh = H @ D.T - A * B", "Rh = H @ D.T - A * A", "test_oracle_codec.py"),
    "grad-D-sign": ("codec", "Rb.T @ V + lam * (Rh.T @ H))", "Rb.T @ V - lam * (Rh.T @ H))",
                    "test_oracle_codec.py"),
    "grad-h-decoder-permuted": ("codec", "Gh = lam * (Rh @ D)", "Gh = lam * (Rh @ D[::-1])",
                                "test_oracle_codec.py"),
    "grad-u-cross-term": ("codec", "Gu = Ra @ D + Gh * V", "Gu = Ra @ D + Gh * U", "test_oracle_codec.py"),
    "eq8-cosine-factor": ("codec", "e2e = (mse * (2.0 - cos)).mean()", "e2e = (mse * (1.0 - cos)).mean()",
                          "test_oracle_codec.py"),
    "eq8-rec-wrong-spectrum": ("codec", "((V @ D.T - B) ** 2).mean()\n", "((V @ D.T - A) ** 2).mean()\n",
                               "test_oracle_codec.py"),
    "eq8-code-normaliser": ("codec", "code = ((H - Tg @ E.T) ** 2).mean()",
                            "code = ((H - Tg @ E.T) ** 2).sum() / H.shape[0]", "test_oracle_codec.py"),
    "eq8-colour-normaliser": ("codec", "col = ((S @ T.T - Tg @ T.T) ** 2).mean()",
                              "col = ((S @ T.T - Tg @ T.T) ** 2).mean() * 3", "test_oracle_codec.py"),
    "eq8-grad-cosine-sign": ("codec", "(2.0 / n) * Rh - M[:, None] * dcos)", "(2.0 / n) * Rh + M[:, None] * dcos)",
                             "test_oracle_codec.py"),
    "eq8-grad-code-sign": ("codec", "Gv.T @ B - lk * (2.0 / k) * (Dc.T @ Tg)) / N",
                           "Gv.T @ B + lk * (2.0 / k) * (Dc.T @ Tg)) / N", "test_oracle_codec.py"),
    "adam-no-bias-correction": ("codec", "m_hat = self.m[i] / (1.0 - self.b1 ** self.t)", "m_hat = self.m[i]",
                                "test_oracle_codec.py"),
    # multi-bounce recurrence (Eq. 10)
    "bounce-restarts-from-light": ("multibounce", "S = R[:, b] * S", "S = R[:, b] * L",
                                   "test_oracle_multibounce.py"),
    "bounce-latent-restarts": ("multibounce", "z = blockwise_product(R[:, b] @ E.T, z)",
                               "z = blockwise_product(R[:, b] @ E.T, L @ E.T)", "test_oracle_multibounce.py"),
    "bounce-cmf-rows-swapped": ("multibounce", "xl.append((z @ D.T) @ T.T)", "xl.append((z @ D.T) @ T[::-1].T)",
                                "test_oracle_multibounce.py"),
    # upsampling network and its training (Sec. 5)
    "silu-negative-branch": ("upsample", "np.where(x >= 0, x / (1.0 + e), x * e / (1.0 + e))",
                             "np.where(x >= 0, x / (1.0 + e), x / (1.0 + e))", "test_oracle_upsample.py"),
    "layer2-bias-dropped": ("upsample", 'h2 = silu(h1 @ _f64(net["W2"]).T + _f64(net["b2"]))',
                            'h2 = silu(h1 @ _f64(net["W2"]).T)', "test_oracle_upsample.py"),
    "maxabs-grad-sign": ("upsample", "dz[np.arange(N), cstar] += w_max", "dz[np.arange(N), cstar] -= w_max",
                         "test_oracle_upsample.py"),
    "dsilu-sign": ("upsample", "return s + x * s * (1.0 - s)", "return s + x * s * (1.0 + s)",
                   "test_oracle_upsample.py"),
    "grad-W2-transposed": ("upsample", "W2=dp2.T @ h1", "W2=(dp2.T @ h1).T", "test_oracle_upsample.py"),
    "lab-b-sign": ("upsample", "200.0 * (f[:, 1] - f[:, 2])", "200.0 * (f[:, 2] - f[:, 1])",
                   "test_oracle_upsample.py"),
    "lab-jacobian-sign": ("upsample", "500.0 * fp[:, 0], -500.0 * fp[:, 1]", "500.0 * fp[:, 0], 500.0 * fp[:, 1]",
                          "test_oracle_upsample.py"),
    "colour-grad-sign": ("upsample", "dz += w_col * gxyz @ M", "dz -= w_col * gxyz @ M", "test_oracle_upsample.py"),
    "adamw-decay-dropped": ("upsample", "w = _f64(w) * (1.0 - self.lr * self.wd)", "w = _f64(w)",
                            "test_oracle_upsample.py"),
    "adamw-no-clipping": ("upsample", "scale = min(1.0, self.max_norm / (norm + 1e-6))", "scale = 1.0",
                          "test_oracle_upsample.py"),
}

ORACLE_MODULES = ("records", "shade", "multibounce", "codec", "upsample")


def install(mid: str):
    """Replace oracle.<module> by its mutated source and re-import the other
    oracle modules so that they bind to it."""
    module, old, new, _ = MUTANTS[mid]
    import oracle
    path = os.path.join(ROOT, "oracle", module + ".py")
    src = open(path).read()
    if src.count(old) != 1:
        raise RuntimeError(f"mutant {mid}: the text to replace occurs {src.count(old)} times in {path}")
    mod = types.ModuleType(f"oracle.{module}")
    mod.__file__, mod.__package__ = path, "oracle"
    sys.modules[mod.__name__] = mod
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    setattr(oracle, module, mod)
    for other in ORACLE_MODULES:
        if other != module:
            setattr(oracle, other, importlib.reload(sys.modules[f"oracle.{other}"]))
