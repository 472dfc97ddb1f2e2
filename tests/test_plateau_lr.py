"""The upsampler fit's reduce-on-plateau rule (Sec. 5.2 schedule) against
torch.optim.lr_scheduler.ReduceLROnPlateau with the same settings, on loss
sequences that improve, stall, improve by less than the threshold and reach
the floor."""

import numpy as np
import pytest
import torch

from paper_2602_18741_amd.upsample_fit import PlateauLR


def _torch_rates(losses, lr, factor, patience, min_lr):
    p = torch.nn.Parameter(torch.zeros(1))
    opt = torch.optim.SGD([p], lr=lr)
    sched = torch.optim.lr_scheduler.ReduceLROnPlateau(opt, mode="min", factor=factor, patience=patience,
                                                       min_lr=min_lr)
    out = []
    for x in losses:
        sched.step(x)
        out.append(opt.param_groups[0]["lr"])
    return out


@pytest.mark.parametrize("patience,factor", [(0, 0.5), (3, 0.5), (7, 0.3), (200, 0.5)])
def test_matches_torch_reduce_on_plateau(patience, factor):
    rng = np.random.default_rng(patience)
    n = 3000
    trend = np.concatenate([np.linspace(1.0, 0.5, 300), np.full(700, 0.5), np.linspace(0.5, 0.49995, 500),
                            np.linspace(0.49, 0.2, 500), np.full(1000, 0.2)])
    losses = (trend * (1 + 0.01 * rng.standard_normal(n))).tolist()
    rule = PlateauLR(2e-3, factor=factor, patience=patience, min_lr=1e-6)
    ours = [rule.step(x) for x in losses]
    ref = _torch_rates(losses, 2e-3, factor, patience, 1e-6)
    assert np.allclose(ours, ref, rtol=1e-12, atol=0)
    assert min(ours) >= 1e-6


def test_floor_and_bad_factor():
    rule = PlateauLR(1e-3, factor=0.5, patience=0, min_lr=2e-4)
    rates = [rule.step(1.0) for _ in range(10)]
    assert rates[0] == 1e-3 and rates[-1] == 2e-4
    with pytest.raises(ValueError):
        PlateauLR(1e-3, factor=1.0)
