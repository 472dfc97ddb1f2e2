"""Fitting the non-negative linear codec on the GPU (Sec. 4.3 objectives).

Each step draws N (reflectance, light) pairs by index from device-resident
pools with the counter-based index generator (the counter base is the Adam
step counter, so a captured graph draws fresh pairs on every replay) inside
hc_codec_step, which also applies the fused Adam update.  The step can be captured
once in a HIP graph and replayed.  State (parameters, Adam moments, step)
round-trips through .npz checkpoints.
"""

from __future__ import annotations

import numpy as np
import torch

from . import ops


class CodecFit:
    def __init__(self, we0: np.ndarray, wd0: np.ndarray, pool_a: torch.Tensor, pool_b: torch.Tensor,
                 batch: int = 65536, lam: float = 1.0, beta: float = 10.0, lr: float = 1e-3,
                 seed: int = 0, dtype=torch.float32, objective: str = "l2", T=None,
                 weights=ops.EQ8_WEIGHTS):
        """objective "l2" (two-term squared error weighted by lam) or "eq8"
        (the four-term loss of Eq. 8 with `weights` and the 3 x n
        colour-matching matrix T)."""
        dev = pool_a.device
        self.k, self.n = we0.shape
        self.N, self.lam, self.beta, self.seed = batch, lam, beta, seed
        self.objective, self.eq8_weights = objective, tuple(float(w) for w in weights)
        self.T = None if T is None else torch.as_tensor(np.asarray(T), dtype=dtype).to(dev).contiguous()
        self.Wt_E = torch.tensor(we0, dtype=dtype, device=dev)
        self.Wt_D = torch.tensor(wd0, dtype=dtype, device=dev)
        self.pool_a = pool_a.to(dtype).contiguous()
        self.pool_b = pool_b.to(dtype).contiguous()
        self.adam = dict(m_E=torch.zeros_like(self.Wt_E), v_E=torch.zeros_like(self.Wt_E),
                         m_D=torch.zeros_like(self.Wt_D), v_D=torch.zeros_like(self.Wt_D),
                         step=torch.zeros(1, dtype=torch.int64, device=dev), lr=lr,
                         beta1=0.9, beta2=0.999, eps=1e-8)
        self.loss = torch.zeros((), dtype=dtype, device=dev)
        self.ws = ops.CodecWorkspace(self.k, self.n, batch, dev)
        self.graph, self.graph_steps = None, 1

    def _step(self):
        # rows for step t: counters [t*N, (t+1)*N) of two seeded index streams
        # (the indices ops.gen_indices would write), drawn inside the step
        draw = dict(seed_a=2 * self.seed + 1, seed_b=2 * self.seed + 2, step=self.adam["step"])
        ops.codec_step(self.Wt_E, self.Wt_D, self.pool_a, self.pool_b, self.N, lam=self.lam,
                       beta=self.beta, draw=draw, loss=self.loss,
                       adam=self.adam, workspace=self.ws, objective=self.objective, T=self.T,
                       weights=self.eq8_weights)

    def capture(self, steps: int = 1):
        """Record `steps` consecutive steps in one HIP graph (run a warm-up step
        first, as graph capture needs the kernels loaded).  Later run() calls
        replay it as often as it fits and take any remaining steps one by one;
        each captured step reads the device step counter when it runs, so every
        replay draws new pairs."""
        if steps < 1:
            raise ValueError("steps must be >= 1")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for _ in range(steps):
                self._step()
        torch.cuda.current_stream().wait_stream(s)
        self.graph, self.graph_steps = g, steps

    def run(self, steps: int):
        if self.graph is not None:
            for _ in range(steps // self.graph_steps):
                self.graph.replay()
            steps %= self.graph_steps
        for _ in range(steps):
            self._step()
        return self.loss

    @property
    def steps_done(self) -> int:
        return int(self.adam["step"].item())

    def weights(self):
        """float32 E = softplus(Wt_E) (k x n) and D = softplus(Wt_D) (n x k)."""
        return ops.codec_weights(self.Wt_E, self.Wt_D, self.beta)

    def state_dict(self) -> dict:
        d = {k: v.detach().cpu().numpy() for k, v in self.adam.items() if torch.is_tensor(v)}
        d.update(Wt_E=self.Wt_E.cpu().numpy(), Wt_D=self.Wt_D.cpu().numpy(),
                 meta=np.array([self.N, self.seed], dtype=np.int64),
                 hyper=np.array([self.lam, self.beta, self.adam["lr"]], dtype=np.float64))
        return d

    def load_state_dict(self, d: dict):
        for name in ("m_E", "v_E", "m_D", "v_D", "step"):
            self.adam[name].copy_(torch.from_numpy(np.asarray(d[name])))
        self.Wt_E.copy_(torch.from_numpy(np.asarray(d["Wt_E"])))
        self.Wt_D.copy_(torch.from_numpy(np.asarray(d["Wt_D"])))

    def save(self, path: str):
        np.savez(path, **self.state_dict())

    def load(self, path: str):
        with np.load(path, allow_pickle=False) as f:
            self.load_state_dict({k: f[k] for k in f.files})
