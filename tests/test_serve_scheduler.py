"""The serving scheduler against a CPU fake backend: coverage of every
pixel, memory budget, FIFO admission, failure injection, interleaving."""

import numpy as np
import pytest

from paper_2602_18741_amd.serve import Request, Scheduler, make_requests, span_tiles


class Handle:
    def __init__(self, polls_needed):
        self.polls = 0
        self.need = polls_needed


class FakeBackend:
    """Records what the scheduler asks for; 'executes' a plan by counting
    which pixels were shaded and decoded."""

    def __init__(self, fail_prepare=(), fail_launch_iteration=None, polls=2, upload_polls=0):
        self.fail_prepare = set(fail_prepare)
        self.fail_launch_iteration = fail_launch_iteration
        self.polls = polls
        self.shaded, self.decoded, self.order = {}, {}, []
        self.live_bytes = 0
        self.max_live = 0
        self.launches = 0
        self.resident = {}          # asset -> [state, polls until arrived]
        self.upload_polls = upload_polls
        self.encoded = []

    def request_bytes(self, req):
        return req.n_pixels * 10

    def prepare(self, req):
        if req.rid in self.fail_prepare:
            raise RuntimeError("injected prepare failure")
        self.asset_of = getattr(self, "asset_of", {})
        self.asset_of[req.rid] = req.asset
        self.shaded[req.rid] = np.zeros(req.n_pixels, np.int32)
        self.decoded[req.rid] = np.zeros(req.n_pixels, np.int32)
        self.live_bytes += self.request_bytes(req)
        self.max_live = max(self.max_live, self.live_bytes)
        self.order.append(req.rid)
        if req.asset not in self.resident:
            self.resident[req.asset] = ["pending", self.upload_polls]

    def asset_state(self, asset):
        a = self.resident[asset]
        if a[0] == "pending":
            if a[1] <= 0:
                a[0] = "needs_encode"
            a[1] -= 1
        return a[0]

    def launch(self, plan):
        self.launches += 1
        if self.fail_launch_iteration == self.launches:
            raise RuntimeError("injected launch failure")
        self.encoded.extend(plan.encode)
        for a in plan.encode:
            self.resident[a][0] = "ready"
        idx, begin, end = span_tiles(plan.shade)
        for i in idx:
            assert self.resident[self.asset_of[plan.shade[i][0]]][0] == "ready", "tile before its asset"
        assert idx.size == plan.n_shade
        for i, b, e in zip(idx, begin, end):
            self.shaded[plan.shade[i][0]][b:e] += 1
        idx, begin, end = span_tiles(plan.decode)
        for i, b, e in zip(idx, begin, end):
            rid = plan.decode[i][0]
            assert (self.shaded[rid][b:e] == 1).all(), "decode before every pixel is shaded"
            self.decoded[rid][b:e] += 1
        return Handle(self.polls)

    def poll(self, h):
        h.polls += 1
        return h.polls >= h.need

    def finish(self, req):
        req.result = (self.shaded[req.rid].copy(), self.decoded[req.rid].copy())

    def release(self, req):
        if req.rid in self.shaded:
            self.live_bytes -= self.request_bytes(req)
            del self.shaded[req.rid], self.decoded[req.rid]


def drive(sched, reqs, max_steps=100000):
    reqs = sorted(reqs, key=lambda r: r.arrival)
    t = 0.0
    i = 0
    for _ in range(max_steps):
        while i < len(reqs) and reqs[i].arrival <= t:
            sched.submit(reqs[i])
            i += 1
        sched.step(t)
        t += 1e-4
        if i == len(reqs) and sched.idle:
            return
    raise AssertionError("scheduler did not drain")


def test_span_expansion():
    idx, b, e = span_tiles([(7, 0, 10, 4), (9, 5, 6, 100), (3, 100, 112, 4)])
    assert idx.tolist() == [0, 0, 0, 1, 2, 2, 2]
    assert b.tolist() == [0, 4, 8, 5, 100, 104, 108]
    assert e.tolist() == [4, 8, 10, 6, 104, 108, 112]


def test_every_pixel_shaded_and_decoded_once():
    be = FakeBackend()
    sched = Scheduler(be, max_frames=8, mem_budget=1e9, tile_pixels=5000, iter_vertices=2e6)
    reqs = make_requests(rate=5000, count=40, n_assets=6, seed=1)
    drive(sched, reqs)
    assert all(r.state == "done" for r in reqs)
    for r in reqs:
        shaded, decoded = r.result
        assert (shaded == 1).all() and (decoded == 1).all()
        assert r.t_admit >= r.arrival and r.t_done >= r.t_admit
    assert sorted(set(be.encoded)) == sorted(set(r.asset for r in reqs))
    assert len(be.encoded) == len(set(be.encoded))        # each asset encoded once
    assert sched.mem_used == 0 and len(sched.free_slots) == 8


def test_memory_budget_and_fifo_admission():
    be = FakeBackend()
    budget = 3 * 1920 * 1080 * 10
    sched = Scheduler(be, max_frames=64, mem_budget=budget, tile_pixels=8192, iter_vertices=5e6)
    reqs = make_requests(rate=1e6, count=30, n_assets=4, seed=2)
    reqs = [r for r in reqs if r.n_pixels * 10 <= budget]
    drive(sched, reqs)
    assert be.max_live <= budget
    assert be.order == sorted(be.order)                   # admitted in arrival order
    assert all(r.state == "done" for r in reqs)


def test_request_over_budget_is_rejected():
    be = FakeBackend()
    sched = Scheduler(be, mem_budget=1000)
    big = Request(rid=0, asset=0, width=100, height=100, spp=1, l_min=1, l_max=1, seed=0)
    sched.submit(big)
    assert big.state == "failed" and "budget" in big.error and sched.rejected == [big]
    assert sched.idle


def test_prepare_failure_frees_slot_and_memory():
    be = FakeBackend(fail_prepare={3, 7})
    sched = Scheduler(be, max_frames=4, mem_budget=1e9, tile_pixels=4096, iter_vertices=1e6)
    reqs = make_requests(rate=1e4, count=12, n_assets=3, seed=3)
    drive(sched, reqs)
    failed = {r.rid for r in reqs if r.state == "failed"}
    assert failed == {3, 7}
    assert all(r.state == "done" for r in reqs if r.rid not in failed)
    assert sched.mem_used == 0 and len(sched.free_slots) == 4 and be.live_bytes == 0


def test_launch_failure_fails_only_its_frames():
    be = FakeBackend(fail_launch_iteration=3)
    sched = Scheduler(be, max_frames=16, mem_budget=1e9, tile_pixels=4096, iter_vertices=3e5)
    reqs = make_requests(rate=2e3, count=10, n_assets=3, seed=4)
    drive(sched, reqs)
    failed = [r for r in reqs if r.state == "failed"]
    assert 1 <= len(failed) < len(reqs)
    assert all("launch" in r.error for r in failed)
    assert all(r.state == "done" for r in reqs if r not in failed)
    assert sched.mem_used == 0 and be.live_bytes == 0


def test_frames_wait_for_their_asset_but_not_for_others():
    """A frame whose asset is still arriving is not tiled; frames with
    resident assets proceed meanwhile."""
    be = FakeBackend(upload_polls=40)
    sched = Scheduler(be, max_frames=8, mem_budget=1e12, tile_pixels=4096, iter_vertices=1e6)
    first = Request(rid=0, asset=0, width=256, height=256, spp=1, l_min=1, l_max=4, seed=0, arrival=0.0)
    drive(sched, [first])
    be.upload_polls = 400
    late = Request(rid=1, asset=1, width=256, height=256, spp=1, l_min=1, l_max=4, seed=1, arrival=1.0)
    warm = Request(rid=2, asset=0, width=256, height=256, spp=1, l_min=1, l_max=4, seed=2, arrival=1.0001)
    drive(sched, [late, warm])
    assert late.state == warm.state == "done"
    assert warm.t_done < late.t_done


def test_small_frame_overtakes_a_large_one():
    """Iteration-level batching: a small frame arriving while a 4K frame is
    being shaded completes first."""
    be = FakeBackend()
    sched = Scheduler(be, max_frames=8, mem_budget=1e12, tile_pixels=4096, iter_vertices=4e6)
    big = Request(rid=0, asset=0, width=3840, height=2160, spp=16, l_min=1, l_max=4, seed=0, arrival=0.0)
    small = Request(rid=1, asset=1, width=256, height=256, spp=1, l_min=1, l_max=4, seed=1,
                    arrival=5e-4)
    drive(sched, [big, small])
    assert big.state == small.state == "done"
    assert small.t_done < big.t_done
    assert sched.iterations > 10
