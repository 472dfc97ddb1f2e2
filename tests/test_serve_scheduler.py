"""The serving scheduler against a CPU fake backend: coverage of every
pixel, memory budget, FIFO admission, failure injection, interleaving."""

import numpy as np
import pytest

from paper_2602_18741_amd.serve import Request, Scheduler, make_requests, span_tiles


class Handle:
    def __init__(self, polls_needed, encode=()):
        self.polls = 0
        self.need = polls_needed
        self.encode = list(encode)


class FakeBackend:
    """Records what the scheduler asks for; 'executes' a plan by counting
    which pixels were shaded and decoded, and tracks the device bytes the
    scheduler has it hold (request buffers and resident assets)."""

    def __init__(self, fail_prepare=(), fail_launch_iteration=None, polls=2, upload_polls=0,
                 asset_size=0.0, staging=0.0, jobs_per_asset=1, max_jobs=4096):
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
        self.asset_size, self.staging = asset_size, staging
        self.jobs_per_asset, self.max_jobs = jobs_per_asset, max_jobs
        self.max_plan_jobs = 0
        self.evicted = []
        self.unstaged = set()       # encoded assets whose staging copy is gone

    def _held(self, delta):
        self.live_bytes += delta
        self.max_live = max(self.max_live, self.live_bytes)

    def iteration_vertices(self):
        return 4e7

    def request_bytes(self, req):
        return req.n_pixels * 10

    def asset_bytes(self, asset, loading):
        return self.asset_size + (self.staging if loading else 0.0)

    def encode_jobs(self, asset):
        return self.jobs_per_asset

    def load_asset(self, asset):
        assert asset not in self.resident
        self.resident[asset] = ["pending", self.upload_polls]
        self._held(self.asset_bytes(asset, True))

    def evict_asset(self, asset):
        assert self.resident[asset][0] != "pending"
        # an asset holds its staging copy until the iteration with its encode ends
        self._held(-self.asset_bytes(asset, asset not in self.unstaged))
        del self.resident[asset]
        self.unstaged.discard(asset)
        self.evicted.append(asset)

    def prepare(self, req):
        if req.rid in self.fail_prepare:
            raise RuntimeError("injected prepare failure")
        assert req.asset in self.resident
        self.asset_of = getattr(self, "asset_of", {})
        self.asset_of[req.rid] = req.asset
        self.shaded[req.rid] = np.zeros(req.n_pixels, np.int32)
        self.decoded[req.rid] = np.zeros(req.n_pixels, np.int32)
        self._held(self.request_bytes(req))
        self.order.append(req.rid)

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
        jobs = sum(self.encode_jobs(a) for a in plan.encode)
        assert jobs <= self.max_jobs
        self.max_plan_jobs = max(self.max_plan_jobs, jobs)
        for a in plan.encode:
            assert self.resident[a][0] == "needs_encode"
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
        return Handle(self.polls, plan.encode)

    def poll(self, h):
        h.polls += 1
        if h.polls < h.need:
            return False
        for a in h.encode:                       # the iteration ended: staging copies go
            if a in self.resident and a not in self.unstaged:
                self.unstaged.add(a)
                self._held(-self.staging)
        return True

    def finish(self, req):
        req.result = (self.shaded[req.rid].copy(), self.decoded[req.rid].copy())

    def release(self, req):
        if req.rid in self.shaded:
            self._held(-self.request_bytes(req))
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
    assert sched.mem_used == be.live_bytes == 0 and len(sched.free_slots) == 8


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


def test_assets_and_frames_share_one_budget_with_back_pressure():
    """Resident assets count against the same budget as frame buffers: with
    room for about two assets beside the frames, unused assets are evicted
    (least recently used first) and the queue waits rather than exceed the
    budget; the scheduler's and the backend's byte counts agree throughout."""
    asset, staging = 2e7, 1e7
    be = FakeBackend(asset_size=asset, staging=staging, upload_polls=3)
    budget = 2 * (asset + staging) + 3 * 1280 * 720 * 10
    sched = Scheduler(be, max_frames=16, mem_budget=budget, tile_pixels=8192, iter_vertices=5e6)
    reqs = [r for r in make_requests(rate=3e3, count=60, n_assets=6, seed=5) if r.n_pixels * 10 <= 2e7]
    t, i = 0.0, 0
    while i < len(reqs) or not sched.idle:
        while i < len(reqs) and reqs[i].arrival <= t:
            sched.submit(reqs[i])
            i += 1
        sched.step(t)
        assert sched.mem_used == pytest.approx(be.live_bytes)
        t += 1e-4
    assert all(r.state == "done" for r in reqs)
    assert be.max_live <= budget and sched.mem_peak <= budget
    assert be.evicted and sched.evictions == len(be.evicted)
    # only assets still resident are charged, at their encoded size
    assert sched.mem_used == pytest.approx(asset * len(sched.assets))


def test_request_that_can_never_fit_is_rejected_and_others_complete():
    be = FakeBackend(asset_size=5e6, staging=5e6)
    sched = Scheduler(be, max_frames=8, mem_budget=1.2e7, tile_pixels=4096, iter_vertices=1e6)
    ok = [Request(rid=i, asset=i % 2, width=256, height=256, spp=1, l_min=1, l_max=2, seed=i,
                  arrival=1e-4 * i) for i in range(4)]
    big = Request(rid=9, asset=0, width=640, height=480, spp=1, l_min=1, l_max=2, seed=9, arrival=2e-4)
    drive(sched, ok + [big])
    assert big.state == "failed" and "budget" in big.error and sched.rejected == [big]
    assert all(r.state == "done" for r in ok)


def test_encode_jobs_past_the_table_are_deferred():
    """Three new assets of two encode jobs each, table of three: one encode
    per iteration, every frame tiled only after its asset's encode."""
    be = FakeBackend(jobs_per_asset=2, max_jobs=3)
    sched = Scheduler(be, max_frames=8, mem_budget=1e9, tile_pixels=4096, iter_vertices=1e6)
    reqs = [Request(rid=i, asset=i, width=256, height=256, spp=1, l_min=1, l_max=2, seed=i, arrival=0.0)
            for i in range(3)]
    drive(sched, reqs)
    assert all(r.state == "done" for r in reqs)
    assert be.max_plan_jobs == 2 and sorted(be.encoded) == [0, 1, 2]


def test_asset_of_a_failed_request_is_evicted_under_pressure():
    """The only request of an asset fails in prepare: the asset (never
    encoded) is evicted when memory is needed."""
    be = FakeBackend(fail_prepare={0}, asset_size=4e6, staging=4e6)
    sched = Scheduler(be, max_frames=8, mem_budget=1.0e7, tile_pixels=4096, iter_vertices=1e6)
    first = Request(rid=0, asset=0, width=64, height=64, spp=1, l_min=1, l_max=1, seed=0, arrival=0.0)
    second = Request(rid=1, asset=1, width=64, height=64, spp=1, l_min=1, l_max=1, seed=1, arrival=1e-3)
    drive(sched, [first, second])
    assert first.state == "failed" and second.state == "done"
    assert be.evicted == [0]
