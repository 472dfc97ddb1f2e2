"""Fitting the RGB-to-latent upsampling network on the GPU (Sec. 5.2).

Each step draws a batch of (RGB, target code) rows by index from
device-resident tables with the counter-based index generator (the counter
base is the optimizer's step counter, so a captured graph draws a fresh
batch on every replay) inside hc_upsample_train_step, which also applies the
fused clipping and AdamW update.  The codec is frozen: the targets are codes of
the training spectra and M = T D maps a code to XYZ for the colour term.
"""

from __future__ import annotations

import numpy as np
import torch

from . import ops


def default_init(k: int, seed: int) -> np.ndarray:
    """Packed parameters with torch.nn.Linear's default initialisation:
    weights and biases uniform in +-1/sqrt(fan_in)."""
    rng = np.random.default_rng(seed)
    h = ops.MLP_HIDDEN
    parts = []
    for fan_in, shape in ((3, (h, 3)), (3, (h,)), (h, (h, h)), (h, (h,)), (h, (k, h)), (h, (k,))):
        b = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, shape).ravel())
    return np.concatenate(parts).astype(np.float32)


def training_pairs(E: torch.Tensor, T: torch.Tensor, spectra: torch.Tensor, n: int):
    """Linear RGB (rows of 4 floats, the 4th 0) and codes (blocked layout) of
    spectra (rows padded to a multiple of 4 floats), both computed by the
    encode kernel: the codes with the codec's encoder, the colours with the
    3 x n matrix XYZ->linear-sRGB times T (the linear RGB of Sec. 5.2)."""
    import synth
    to_rgb = torch.from_numpy((synth.XYZ_TO_LINEAR_SRGB @ T.cpu().double().numpy()).astype(np.float32))
    rgb = ops.encode(to_rgb.to(spectra.device), spectra, n=n)
    z = ops.encode(E, spectra, n=n)
    return rgb, z


class PlateauLR:
    """Reduce-on-plateau learning-rate rule (the schedule of Sec. 5.2: factor
    0.5, patience 200, floor 1e-6), in the form of torch's ReduceLROnPlateau
    with its defaults otherwise: a loss counts as better when it is below the
    best so far by more than `threshold` relative; after more than `patience`
    evaluations without one the rate is multiplied by `factor`, not below
    `min_lr` (changes smaller than `eps` are skipped), and the count restarts."""

    def __init__(self, lr: float, factor: float = 0.5, patience: int = 200, min_lr: float = 1e-6,
                 threshold: float = 1e-4, eps: float = 1e-8):
        if not 0.0 < factor < 1.0:
            raise ValueError("factor must be in (0, 1)")
        self.lr, self.factor, self.patience = float(lr), float(factor), int(patience)
        self.min_lr, self.threshold, self.eps = float(min_lr), float(threshold), float(eps)
        self.best = float("inf")
        self.bad = 0

    def step(self, loss: float) -> float:
        loss = float(loss)
        if loss < self.best * (1.0 - self.threshold):
            self.best, self.bad = loss, 0
        else:
            self.bad += 1
        if self.bad > self.patience:
            new = max(self.lr * self.factor, self.min_lr)
            if self.lr - new > self.eps:
                self.lr = new
            self.bad = 0
        return self.lr


class UpsampleFit:
    def __init__(self, rgb: torch.Tensor, z_gt: torch.Tensor, M: torch.Tensor, white, k: int,
                 batch: int = 1024, lr: float = 2e-3, weight_decay: float = 1e-5,
                 max_grad_norm: float = 1.0, w_max: float = 0.3, w_col: float = 0.05, seed: int = 0,
                 init_seed: int = 0):
        dev = rgb.device
        self.k, self.N, self.seed = k, batch, seed
        self.rgb, self.z_gt, self.M = rgb, z_gt, M.contiguous()
        self.white = tuple(float(w) for w in white)
        self.w_max, self.w_col = w_max, w_col
        self.params = torch.from_numpy(default_init(k, init_seed)).to(dev)
        self.opt = dict(m=torch.zeros_like(self.params), v=torch.zeros_like(self.params),
                        step=torch.zeros(1, dtype=torch.int64, device=dev), lr=lr, beta1=0.9,
                        beta2=0.999, eps=1e-8, weight_decay=weight_decay,
                        max_grad_norm=max_grad_norm)
        self.loss = torch.zeros((), dtype=torch.float32, device=dev)
        self.ws = ops.UpsampleWorkspace(k, batch, dev)
        self.graph, self.graph_steps = None, 1

    def _step(self):
        # rows for step t: counters [t*N, (t+1)*N) of a seeded index stream
        # (the indices ops.gen_indices would write), drawn inside the step
        ops.upsample_train_step(self.params, self.rgb, self.z_gt, self.M, self.white, self.k, self.N,
                                draw=dict(seed=2 * self.seed + 7, step=self.opt["step"]), w_max=self.w_max,
                                w_col=self.w_col, loss=self.loss, opt=self.opt, workspace=self.ws)

    def capture(self, steps: int = 1):
        """Record `steps` consecutive steps in one HIP graph (run a warm-up step
        first, as graph capture needs the kernels loaded).  Later run() calls
        replay it as often as it fits and take any remaining steps one by one;
        each captured step reads the device step counter when it runs, so every
        replay draws a new batch."""
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

    def run_epochs(self, epochs: int, epoch_steps: int, plateau: PlateauLR | None = None):
        """`epochs` rounds of `epoch_steps` steps; after each, the plateau rule
        (if any) sees the loss of the round's last batch and may lower the
        learning rate.  The rate is a launch argument, so a captured graph is
        recorded again when it changes.  Returns the per-round losses."""
        losses = []
        for _ in range(epochs):
            loss = float(self.run(epoch_steps))
            losses.append(loss)
            if plateau is not None:
                lr = plateau.step(loss)
                if lr != self.opt["lr"]:
                    self.opt["lr"] = lr
                    if self.graph is not None:
                        self.capture(self.graph_steps)
        return losses

    @property
    def steps_done(self) -> int:
        return int(self.opt["step"].item())

    def net(self) -> dict:
        """W1, b1, W2, b2, W3, b3 views of the packed parameters (for ops.upsample)."""
        return {name: v.contiguous() for name, v in ops.unpack_mlp(self.params, self.k).items()}
