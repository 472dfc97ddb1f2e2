"""The random-gather probe reads what it is given: the sum of its per-lane
outputs is sum_v w_v * (sum of the row's first whole 16-byte chunks covering
row_floats floats, row t_v), for every issue shape, with records past the
table clamped to its last row."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("row_floats,ld,lanes", [(8, 8, 1), (12, 16, 1), (16, 16, 1), (31, 32, 8),
                                                 (84, 96, 8), (128, 128, 8)])
@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
def test_probe_sums_the_gathered_rows(gpu, row_floats, ld, lanes, unroll):
    from paper_2602_18741_amd import ops
    rng = np.random.default_rng(row_floats * 10 + unroll)
    rows, nv = 5000, 100_003
    table = rng.uniform(-1, 1, (rows, ld)).astype(np.float32)
    tex = rng.integers(0, rows + 50, nv).astype(np.uint32)         # some past the table
    w = rng.uniform(0, 1, nv).astype(np.float32)
    vtx = np.stack([tex, w.view(np.uint32)], axis=1)
    out = ops.gather_probe(torch.from_numpy(vtx.view(np.int32)).to(gpu), torch.from_numpy(table).to(gpu),
                           row_floats, unroll=unroll, lanes_per_row=lanes, grid=37)
    used = 4 * -(-row_floats // 4)
    rs = table[:, :used].astype(np.float64).sum(axis=1)
    want = (w.astype(np.float64) * rs[np.minimum(tex, rows - 1)]).sum()
    got = out.double().sum().item()
    bound = 1e-5 * (np.abs(w.astype(np.float64) * np.abs(table[:, :used]).sum(axis=1)[
        np.minimum(tex, rows - 1)]).sum())
    assert abs(got - want) <= bound


def test_probe_of_no_records_writes_zeros(gpu):
    from paper_2602_18741_amd import ops
    table = torch.ones(4, 8, device=gpu)
    out = ops.gather_probe(torch.zeros(0, 2, dtype=torch.int32, device=gpu), table, 8, grid=3)
    assert torch.equal(out, torch.zeros_like(out))


@pytest.mark.parametrize("grid", [1, 37, 1024])
def test_stream_probe_reads_and_copies_everything(gpu, grid):
    """Streaming probe: the per-lane sums of the read mode add up to the sum
    of the data (integer values: every partial sum is exact), and the copy
    mode reproduces the source bit for bit, with a ragged tail of chunks."""
    from paper_2602_18741_amd import ops
    rng = np.random.default_rng(grid)
    n16 = 250_003
    src = torch.from_numpy(rng.integers(0, 8, 4 * n16).astype(np.float32)).to(gpu)
    sums = torch.empty(grid * 256, device=gpu)
    ops.stream_probe(src, sums, "read", grid)
    assert sums.double().sum().item() == src.double().sum().item()
    dst = torch.full_like(src, -1.0)
    ops.stream_probe(src, dst, "copy", grid)
    assert torch.equal(dst, src)


def test_alu_probe_fma_chains_and_every_lane(gpu):
    """Issue-rate probe: the multiply-add kind leaves each lane the sum of its
    8 chains x <- 0.999 x + 0.001 (2048 steps from x0 = (lane + i) / 1000)
    plus the untouched fp16 seeds, as the host computes them; every kind
    writes every lane (no NaN left from the fill)."""
    from paper_2602_18741_amd import ops
    grid = 3
    out = torch.full((grid * 256,), float("nan"), device=gpu)
    ops.alu_probe("fma_f32", out)
    lane = np.arange(256, dtype=np.float64)
    want = np.zeros(256)
    for i in range(ops.ALU_PROBE_CHAINS):
        x0 = ((lane + i) * np.float32(1e-3)).astype(np.float32)
        h = x0.astype(np.float16).astype(np.float64)
        ph = (np.float32(0.5) * x0).astype(np.float16).astype(np.float64)
        x = 1.0 - (1.0 - x0.astype(np.float64)) * 0.999 ** ops.ALU_PROBE_ITERS
        want += x + h + h + ph
    got = out.double().cpu().numpy().reshape(grid, 256)
    assert np.abs(got - want).max() <= 1e-3
    for op in ops.ALU_PROBE_OPS[1:]:
        out.fill_(float("nan"))
        ops.alu_probe(op, out)
        torch.cuda.synchronize()
        assert not torch.isnan(out).any(), op
