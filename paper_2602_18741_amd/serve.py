"""Continuous-batching frame server.

Frames arrive as a stream of requests of mixed resolution, samples per pixel
and path length.  The scheduler admits them while frame slots and a device
memory budget allow (FIFO), keeps encoded assets resident across requests
(encode on first use), and runs *iterations*: each iteration shades a
bounded number of pixel tiles taken from all admitted frames, so a request
that arrives while a large frame is in flight joins the next iteration
instead of waiting for that frame to finish.  The latent form decodes each
pixel in the launch that shades it; with a separate decode launch, frames
whose last tile is in an iteration are decoded in the same iteration.

On the GPU an iteration is one replay of a captured HIP graph holding the
table-driven launches (latent form: encode, then shading with the per-pixel
decode in its epilogue, or a separate decode launch); the host only rewrites the
small frame / tile / job tables (copied to the device before the replay) and
launches the per-request path generators.  Up to two iterations are in
flight, so table building overlaps device work.

`Scheduler` holds the policy and is independent of the device; `GpuBackend`
executes plans with libhc; tests drive the scheduler with a CPU fake backend.
"""

from __future__ import annotations

import collections
import ctypes as C
import math
import time
from dataclasses import dataclass, field

import numpy as np


# ------------------------------------------------------------------ requests

@dataclass
class Request:
    rid: int
    asset: int
    width: int
    height: int
    spp: int
    l_min: int
    l_max: int
    seed: int
    arrival: float = 0.0
    keep_result: bool = False
    # filled in by the server
    state: str = "queued"        # queued -> active -> done | failed
    next_pixel: int = 0          # first pixel not yet scheduled
    t_admit: float = math.nan
    t_done: float = math.nan
    error: str | None = None
    result: object = None
    slot: int = -1
    first_use: bool = False      # its admission brought the asset in

    @property
    def n_pixels(self) -> int:
        return self.width * self.height

    @property
    def expected_vertices(self) -> float:
        return self.n_pixels * self.spp * 0.5 * (self.l_min + self.l_max)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclass
class Plan:
    """One iteration: assets to encode, shade tiles, decode tiles, frames
    that complete when the iteration does."""
    encode: list = field(default_factory=list)          # asset ids
    shade: list = field(default_factory=list)           # spans (rid, begin, end, tile)
    decode: list = field(default_factory=list)          # spans (rid, begin, end, tile)
    finishing: list = field(default_factory=list)       # requests
    n_shade: int = 0                                    # tiles in the shade spans


def span_tiles(spans):
    """Expand spans (rid, begin, end, tile) into arrays (span index, begin,
    end) of tiles [b, min(b + tile, end)) for b = begin, begin + tile, ..."""
    if not spans:
        z = np.zeros(0, np.int64)
        return z, z, z
    sp = np.array([(b, e, t) for _, b, e, t in spans], dtype=np.int64)
    counts = -(-(sp[:, 1] - sp[:, 0]) // sp[:, 2])
    idx = np.repeat(np.arange(len(spans)), counts)
    first = np.repeat(np.cumsum(counts) - counts, counts)
    begin = sp[idx, 0] + (np.arange(idx.size) - first) * sp[idx, 2]
    end = np.minimum(begin + sp[idx, 2], sp[idx, 1])
    return idx, begin, end


class Scheduler:
    """Admission, asset residency, tiling and completion bookkeeping (device
    independent).

    One memory budget covers both the admitted requests' buffers and the
    resident assets.  The head of the queue is admitted when its buffers,
    plus its asset if that is not resident, fit the budget, after evicting
    least-recently-used assets that no admitted request uses; otherwise it
    waits (back-pressure) and so does everything behind it (FIFO).  A request
    that could never fit, even with every asset evicted, is rejected at
    submission.

    backend must provide: iteration_vertices() (path-vertices of an
    iteration when the caller gives none); request_bytes(req); asset_bytes(asset, loading)
    (device bytes of a resident asset, and while it is being brought in);
    load_asset(asset) (start bringing it in); evict_asset(asset);
    asset_state(asset) -> "pending" (still arriving), "needs_encode" or
    "ready"; encode_jobs(asset) (encode-table entries of its encode) and
    max_jobs; prepare(req) (allocate, make the records); launch(plan) ->
    handle; poll(handle) -> bool; release(req); finish(req) (fetch results if
    kept).  A frame is tiled only once its asset has arrived (and is encoded
    in that iteration or before), so uploads overlap the shading of other
    frames.  mem_budget None asks the backend (memory_budget()).
    """

    def __init__(self, backend, max_frames: int = 64, mem_budget: float | None = None,
                 tile_pixels: int | None = None, iter_vertices: float | None = None, max_inflight: int = 2,
                 max_tiles: int = 8192, decode_pixels: int = 65536, target_tiles: int = 4096):
        self.b = backend
        self.max_frames = max_frames
        self.mem_budget = float(backend.memory_budget() if mem_budget is None else mem_budget)
        # tile_pixels fixes the tile size; by default each frame's tiles hold
        # about iter_vertices / target_tiles path-vertices, so an iteration
        # carries enough tiles to occupy every workgroup of the launch
        self.tile_pixels = tile_pixels
        self.target_tiles = target_tiles
        # path-vertices per iteration: by default what the backend shades in
        # about the same device time whatever the form (iteration_vertices())
        self.iter_vertices = float(backend.iteration_vertices() if iter_vertices is None else iter_vertices)
        self.max_inflight = max_inflight
        self.max_tiles = max_tiles
        self.decode_pixels = decode_pixels  # decode tiles are larger: 64 frames x 4K fit one table
        self.queue: collections.deque[Request] = collections.deque()
        self.active: list[Request] = []
        self.free_slots = list(range(max_frames))[::-1]
        self.mem_used = 0.0
        self.mem_peak = 0.0
        # resident assets in least-recently-used order: asset -> [refs, bytes charged]
        self.assets: collections.OrderedDict[int, list] = collections.OrderedDict()
        self.inflight: collections.deque = collections.deque()
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.iterations = 0
        self.evictions = 0

    # -------------------------------------------------------------- intake
    def submit(self, req: Request):
        need = self.b.request_bytes(req) + self.b.asset_bytes(req.asset, True)
        if need > self.mem_budget:
            req.state, req.error = "failed", "request larger than the memory budget"
            req.t_done = req.arrival
            self.rejected.append(req)
            return
        self.queue.append(req)

    def _charge(self, nbytes: float):
        self.mem_used += nbytes
        self.mem_peak = max(self.mem_peak, self.mem_used)

    def _evict_for(self, need: float) -> bool:
        """Evict assets no admitted request uses, least recently used first,
        until `need` more bytes fit; True if they do.  An asset still
        arriving is not evicted; one waiting for its encode with no request
        left is (no plan encodes an asset without a request)."""
        for aid in list(self.assets):
            if self.mem_used + need <= self.mem_budget:
                break
            refs, nbytes = self.assets[aid]
            if refs == 0 and self.b.asset_state(aid) != "pending":
                self.b.evict_asset(aid)
                del self.assets[aid]
                self.mem_used -= nbytes
                self.evictions += 1
        return self.mem_used + need <= self.mem_budget

    def _admit(self, now: float):
        while self.queue and self.free_slots:
            req = self.queue[0]
            need = self.b.request_bytes(req)
            new_asset = req.asset not in self.assets
            asset_need = self.b.asset_bytes(req.asset, True) if new_asset else 0.0
            if not self._evict_for(need + asset_need):
                break  # FIFO: the head waits for memory, later requests wait behind it
            self.queue.popleft()
            req.slot = self.free_slots.pop()
            req.t_admit = now
            self._charge(need)
            if new_asset:
                try:
                    self.b.load_asset(req.asset)
                except Exception as e:  # noqa: BLE001 - a failed request must not stop the server
                    self.mem_used -= need
                    self.free_slots.append(req.slot)
                    req.state, req.error, req.t_done = "failed", f"load: {e}", now
                    self.done.append(req)
                    continue
                self.assets[req.asset] = [0, asset_need]
                self._charge(asset_need)
                req.first_use = True
            self.assets.move_to_end(req.asset)
            self.assets[req.asset][0] += 1
            try:
                self.b.prepare(req)
            except Exception as e:  # noqa: BLE001
                self._fail(req, f"prepare: {e}")
                continue
            req.state = "active"
            self.active.append(req)

    def _release(self, req: Request):
        self.b.release(req)
        self.mem_used -= self.b.request_bytes(req)
        self.free_slots.append(req.slot)
        self.assets[req.asset][0] -= 1

    def _fail(self, req: Request, msg: str):
        req.state, req.error = "failed", msg
        req.t_done = time.perf_counter()
        try:
            self._release(req)
        finally:
            if req in self.active:
                self.active.remove(req)
            self.done.append(req)

    # -------------------------------------------------------------- iterations
    def _plan(self) -> Plan | None:
        """Tiles for the next iteration.  Every admitted frame whose asset
        has arrived and that has pixels left gets one tile (so none starves);
        the rest of the vertex budget goes to frames in order of least
        remaining work, which lets small frames finish quickly beside large
        ones.  Assets that arrived since the last iteration are encoded first
        in the same iteration."""
        state = {a: self.b.asset_state(a) for a in {r.asset for r in self.active}}
        plan = Plan()
        jobs = 0
        for a in sorted(a for a, st in state.items() if st == "needs_encode"):
            nj = self.b.encode_jobs(a)
            if jobs + nj > self.b.max_jobs:
                continue        # encoded in a later iteration; its frames wait until then
            plan.encode.append(a)
            jobs += nj
        todo = [r for r in self.active if r.next_pixel < r.n_pixels
                and (state[r.asset] == "ready" or r.asset in plan.encode)]
        per_px = {r.rid: r.spp * 0.5 * (r.l_min + r.l_max) for r in todo}
        todo.sort(key=lambda r: ((r.n_pixels - r.next_pixel) * per_px[r.rid], r.arrival))
        budget = self.iter_vertices
        start = {r.rid: r.next_pixel for r in todo}
        tiles = 0

        def take(req, n_tiles):
            nonlocal budget, tiles
            t = self._tile(req)
            b = req.next_pixel
            e = min(req.n_pixels, b + n_tiles * t)
            req.next_pixel = e
            got = -(-(e - b) // t)
            tiles += got
            budget -= (e - b) * per_px[req.rid]

        for req in todo:
            if tiles >= self.max_tiles:
                break
            take(req, 1)
        for req in todo:
            if budget <= 0 or tiles >= self.max_tiles:
                break
            left = req.n_pixels - req.next_pixel
            if left <= 0:
                continue
            t = self._tile(req)
            want = -(-min(left, int(budget / per_px[req.rid]) + 1) // t)
            take(req, max(1, min(want, self.max_tiles - tiles)))
        for req in todo:
            if req.next_pixel > start[req.rid]:
                plan.shade.append((req.rid, start[req.rid], req.next_pixel, self._tile(req)))
            if req.next_pixel >= req.n_pixels:
                plan.finishing.append(req)
                plan.decode.append((req.rid, 0, req.n_pixels, self.decode_pixels))
        plan.n_shade = tiles
        if not plan.shade and not plan.encode:
            return None
        return plan

    def _tile(self, req) -> int:
        if self.tile_pixels:
            return self.tile_pixels
        per_px = req.spp * 0.5 * (req.l_min + req.l_max)
        px = self.iter_vertices / self.target_tiles / max(per_px, 1.0)
        return int(min(65536, max(256, 256 * round(px / 256))))

    def _complete(self, now: float):
        while self.inflight and self.b.poll(self.inflight[0][0]):
            _, plan = self.inflight.popleft()
            for aid in plan.encode:
                # encoded: the asset's staging copy is gone, only its codes stay
                if aid in self.assets:
                    resident = self.b.asset_bytes(aid, False)
                    self.mem_used -= self.assets[aid][1] - resident
                    self.assets[aid][1] = resident
            for req in plan.finishing:
                if req.state != "active":
                    continue
                req.t_done = now
                try:
                    self.b.finish(req)
                    req.state = "done"
                except Exception as e:  # noqa: BLE001
                    req.state, req.error = "failed", f"finish: {e}"
                self._release(req)
                self.active.remove(req)
                self.done.append(req)

    def step(self, now: float | None = None) -> bool:
        """One scheduling round; returns True if anything happened."""
        now = time.perf_counter() if now is None else now
        before = (len(self.done), len(self.inflight), len(self.queue))
        self._complete(now)
        if len(self.inflight) < self.max_inflight:
            self._admit(now)
            plan = self._plan()
            if plan is not None:
                try:
                    handle = self.b.launch(plan)
                except Exception as e:  # noqa: BLE001
                    for req in list(self.active):
                        if any(sp[0] == req.rid for sp in plan.shade):
                            self._fail(req, f"launch: {e}")
                    return True
                self.inflight.append((handle, plan))
                self.iterations += 1
        return before != (len(self.done), len(self.inflight), len(self.queue))

    @property
    def idle(self) -> bool:
        return not (self.queue or self.active or self.inflight)


# ------------------------------------------------------------------ GPU backend

class _Range:
    """A named range on the host timeline (roctx through torch.cuda.nvtx) for
    profiler marker traces; does nothing when torch has no marker support."""

    def __init__(self, torch, name: str):
        nvtx = getattr(torch.cuda, "nvtx", None)
        self.push = getattr(nvtx, "range_push", None)
        self.pop = getattr(nvtx, "range_pop", None)
        self.name = name

    def __enter__(self):
        if self.push is not None:
            try:
                self.push(self.name)
            except RuntimeError:
                self.push = self.pop = None
        return self

    def __exit__(self, *exc):
        if self.pop is not None:
            self.pop()
        return False


class GpuBackend:
    """Executes plans with the table-driven libhc launches, one captured
    graph per form.  form: "latent" (encode -> shade -> decode) or
    "spectral" (shade straight to XYZ).  In the latent form fused_decode
    (the default) decodes each shaded pixel in the shading launch with the
    decoder matrix M = T D, formed once here: no latent image is kept and
    the plan's decode tiles are not needed; fused_decode=False keeps the
    latent images and runs the decode launch over them (same bits)."""

    JOB_ROWS = 2048          # spectra rows per encode-table entry: a 2048^2 asset spreads over 2,048 workgroups

    def __init__(self, assets, lights, T, E=None, D=None, form: str = "latent", max_frames: int = 64,
                 max_tiles: int = 8192, max_jobs: int = 8192, grid: int = 0, device="cuda",
                 use_graph: bool = True, reserve: float = 0.1, fused_decode: bool = True):
        import torch

        from . import ops
        from ._lib import Frame, Tile, EncodeJob, check, load
        self.torch, self.ops, self.check, self.lib = torch, ops, check, load()
        self.Frame, self.Tile, self.EncodeJob = Frame, Tile, EncodeJob
        self.dev = torch.device(device)
        self.form = form
        self.fused = fused_decode and form == "latent"
        self.assets = assets              # list of pinned host float32 (texels, ld) tensors
        self.n = T.shape[1]
        self.k = E.shape[0] if E is not None else 0
        self.T = T.to(self.dev).contiguous()
        self.E = None if E is None else E.to(self.dev).contiguous()
        self.D = None if D is None else D.to(self.dev).contiguous()
        self.max_frames, self.max_tiles, self.max_jobs, self.grid = max_frames, max_tiles, max_jobs, grid
        self.stream = torch.cuda.Stream(device=self.dev)
        self.copy_stream = torch.cuda.Stream(device=self.dev)   # asset uploads
        lights_d = ops.padded(lights.to(self.dev))
        with torch.cuda.stream(self.stream):
            if form == "latent":
                self.lights = torch.empty(lights.shape[0], ops.latent_width(self.k), device=self.dev)
                ops.encode(self.E, lights_d, n=self.n, out=self.lights)
                self.M = ops.decode_matrix(self.D, self.T, self.k)
            else:
                self.lights = lights_d
        self.stream.synchronize()
        # device tables, and two pinned host copies used alternately
        fb, tb, jb = C.sizeof(Frame), C.sizeof(Tile), C.sizeof(EncodeJob)
        self.sizes = (max_frames * fb, max_tiles * tb, max_tiles * tb, max_jobs * jb, 16)
        total = sum(self.sizes)
        self.d_tables = torch.zeros(total, dtype=torch.uint8, device=self.dev)
        self.h_tables = [torch.zeros(total, dtype=torch.uint8).pin_memory() for _ in range(2)]
        self.h_events = [None, None]
        self.flip = 0
        offs = np.cumsum([0, *self.sizes])
        base = self.d_tables.data_ptr()
        self.d_frames, self.d_tiles, self.d_dtiles, self.d_jobs, self.d_counts = (
            base + int(o) for o in offs[:5])
        self.offs = offs
        self.frames = (Frame * max_frames)()
        self.reqs: dict[int, object] = {}
        # asset id -> {"state", "event", "spectral", "tex"}; "tex" is what the
        # frames read (latent codes, or the spectral rows themselves)
        self.resident: dict[int, dict] = {}
        self.reserve = reserve
        self.pending_free = {}            # handle -> tensors kept alive until the iteration ends
        self.graph = None
        if use_graph:
            self._capture()

    # -------------------------------------------------------------- launches
    def _launch_tables(self):
        i32 = C.c_int32
        st = self.stream.cuda_stream
        cnt = self.d_counts
        if self.form == "latent":
            self.check(self.lib.hc_encode_jobs(self.d_jobs, cnt + 8, self.max_jobs, self.E.data_ptr(),
                                               self.k, self.n, self.grid, st), "hc_encode_jobs")
            if self.fused:
                self.check(self.lib.hc_shade_latent_xyz_tiles(self.d_frames, self.max_frames, self.d_tiles, cnt,
                                                              self.max_tiles, self.k, self.M.data_ptr(),
                                                              self.grid, st), "hc_shade_latent_xyz_tiles")
            else:
                self.check(self.lib.hc_shade_latent_tiles(self.d_frames, self.max_frames, self.d_tiles, cnt,
                                                          self.max_tiles, self.k, self.grid, st),
                           "hc_shade_latent_tiles")
                self.check(self.lib.hc_decode_tiles(self.d_frames, self.max_frames, self.d_dtiles, cnt + 4,
                                                    self.max_tiles, self.D.data_ptr(), self.n, self.k,
                                                    self.T.data_ptr(), self.grid, st), "hc_decode_tiles")
        else:
            self.check(self.lib.hc_shade_spectral_tiles(self.d_frames, self.max_frames, self.d_tiles, cnt,
                                                        self.max_tiles, self.n, self.T.data_ptr(),
                                                        self.grid, st), "hc_shade_spectral_tiles")
        del i32

    def _capture(self):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self._launch_tables()          # warm-up with all counts zero
        self.stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            self._launch_tables()
        self.graph = g

    # -------------------------------------------------------------- scheduler hooks
    ITER_LINES = 40e6        # texel-row cache lines one iteration gathers (about 0.7 ms)

    def iteration_vertices(self) -> float:
        """Path-vertices per iteration.  The shading kernels run at the rate
        of random 128-byte line fetches, one per line of a texel row, so an
        iteration is sized in lines: a k <= 9 code or an n = 31 spectrum is
        one line, an n = 81 spectrum three."""
        row = 4 * (self.ops.latent_width(self.k) if self.form == "latent" else self.ops.line_stride(self.n))
        return self.ITER_LINES / max(1, -(-row // 128))

    def memory_budget(self) -> float:
        """Device memory the scheduler may hand out: what the device has free
        now (with this backend's tables, lights and graph allocated), less a
        reserve fraction for the caching allocator's rounding and
        fragmentation and the path generators' workspaces."""
        cuda = self.torch.cuda
        free, _ = cuda.mem_get_info(self.dev)
        # blocks the caching allocator holds but no tensor uses are free to us
        free += cuda.memory_reserved(self.dev) - cuda.memory_allocated(self.dev)
        return max(0.0, (1.0 - self.reserve) * free - 1e9)

    def request_bytes(self, req) -> float:
        paths = req.n_pixels * req.spp * (4 + 8 * req.l_max) + 4 * req.n_pixels
        # XYZ, plus the latent image when the decode is a launch of its own
        image = 4 * self.ops.latent_width(self.k) if self.form == "latent" and not self.fused else 0
        out = req.n_pixels * (12 + image)
        return float(paths + out + 4096)

    def asset_bytes(self, asset, loading: bool) -> float:
        """Device bytes of an asset: its spectral rows while they arrive and
        wait for the encode (latent form) plus the codes; the codes alone
        once encoded.  The spectral form keeps the rows themselves."""
        host = self.assets[asset]
        spectral = float(host.shape[0] * host.shape[1] * 4)
        if self.form != "latent":
            return spectral
        codes = float(host.shape[0] * 4 * self.ops.line_stride(self.ops.latent_width(self.k)))
        return codes + (spectral if loading else 0.0)

    def encode_jobs(self, asset) -> int:
        return -(-self.assets[asset].shape[0] // self.JOB_ROWS) if self.form == "latent" else 0

    def load_asset(self, asset):
        """Start the upload of an asset (copy stream); the latent form also
        allocates its codes, written by the encode of a later iteration."""
        torch, ops = self.torch, self.ops
        host = self.assets[asset]
        if self.encode_jobs(asset) > self.max_jobs:
            raise RuntimeError(f"asset {asset} needs more encode jobs than the table holds")
        with torch.cuda.stream(self.copy_stream):
            spectral = host.to(self.dev, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        spectral.record_stream(self.stream)
        if self.form == "latent":
            with torch.cuda.stream(self.stream):
                # line-aligned rows: a code never straddles two 128-byte lines
                tex = torch.empty(host.shape[0], ops.line_stride(ops.latent_width(self.k)), device=self.dev)
        else:
            tex = spectral
        self.resident[asset] = dict(state="pending", event=ev, spectral=spectral, tex=tex)

    def evict_asset(self, asset):
        """Drop the device copy of an asset no admitted frame uses.  Its
        memory returns to the allocator pool of the stream it was made on, so
        work still in flight that read it stays ordered before any reuse."""
        del self.resident[asset]

    def prepare(self, req):
        with _Range(self.torch, f"prepare {req.width}x{req.height}x{req.spp}"):
            self._prepare(req)

    def _prepare(self, req):
        torch, ops = self.torch, self.ops
        tex = self.resident[req.asset]["tex"]
        with torch.cuda.stream(self.stream):
            P = ops.Paths(torch.empty(req.n_pixels * req.spp, dtype=torch.int32, device=self.dev),
                          torch.empty(req.n_pixels, dtype=torch.int32, device=self.dev),
                          torch.empty(max(1, req.n_pixels * req.spp * req.l_max), 2, dtype=torch.int32,
                                      device=self.dev), req.n_pixels, req.spp)
            g = self._gen(req, P, tex.shape[0])
            image = (torch.empty(req.n_pixels, ops.latent_width(self.k), device=self.dev)
                     if self.form == "latent" and not self.fused else None)
            xyz = torch.empty(req.n_pixels, 3, device=self.dev)
        f = self.frames[req.slot]
        f.hdr, f.pix_first, f.vtx = P.hdr.data_ptr(), P.pix_first.data_ptr(), P.vtx.data_ptr()
        f.n_pixels, f.n_vertices, f.spp = req.n_pixels, P.vtx.shape[0], req.spp
        f.n_illum, f.tex, f.n_texels, f.ld_tex = self.lights.shape[0], tex.data_ptr(), tex.shape[0], tex.stride(0)
        f.lights, f.ld_lights = self.lights.data_ptr(), self.lights.stride(0)
        f.image, f.ld_image = (image.data_ptr(), image.stride(0)) if image is not None else (None, 0)
        f.xyz = xyz.data_ptr()
        self.reqs[req.rid] = dict(P=P, image=image, xyz=xyz, gen=g, slot=req.slot)

    def asset_state(self, asset) -> str:
        a = self.resident[asset]
        if a["state"] == "pending" and a["event"].query():
            a["state"] = "needs_encode" if self.form == "latent" else "ready"
            if self.form != "latent":
                a["spectral"] = None
        return a["state"]

    def _gen(self, req, P, n_tex):
        from ._lib import PathGen
        g = PathGen(req.n_pixels, req.spp, req.l_min, req.l_max, self.lights.shape[0], n_tex, req.seed)
        wsb = int(self.lib.hc_gen_workspace_size(req.n_pixels))
        ws = self.torch.empty(max(8, wsb), dtype=self.torch.uint8, device=self.dev)
        total = self.torch.empty(1, dtype=self.torch.int64, device=self.dev)
        st = self.stream.cuda_stream
        self.check(self.lib.hc_gen_path_headers(C.byref(g), P.hdr.data_ptr(), P.pix_first.data_ptr(),
                                                total.data_ptr(), ws.data_ptr(), wsb, st),
                   "hc_gen_path_headers")
        self.check(self.lib.hc_gen_path_vertices(C.byref(g), P.pix_first.data_ptr(), P.vtx.data_ptr(),
                                                 P.vtx.shape[0], st), "hc_gen_path_vertices")
        return (ws, total)

    def launch(self, plan):
        with _Range(self.torch, "launch iteration"):
            return self._launch(plan)

    def _launch(self, plan):
        torch = self.torch
        h = self.h_tables[self.flip]
        if self.h_events[self.flip] is not None:
            self.h_events[self.flip].synchronize()   # the copy that last read this buffer is done
        # every table is checked against its capacity before anything is
        # written or any asset changes state, so a refused plan leaves the
        # backend as it was
        parts = []
        for aid in plan.encode:
            a = self.resident[aid]
            spectral, tex = a["spectral"], a["tex"]
            b = np.arange(0, spectral.shape[0], self.JOB_ROWS, dtype=np.int64)
            j = np.zeros(b.size, self._JOB_DT)
            j["S"], j["Z"] = spectral.data_ptr(), tex.data_ptr()
            j["ld_s"], j["ld_z"] = spectral.stride(0), tex.stride(0)
            j["begin"], j["end"] = b, np.minimum(b + self.JOB_ROWS, spectral.shape[0])
            parts.append(j)
        jobs = np.concatenate(parts) if parts else np.zeros(0, self._JOB_DT)
        if jobs.size > self.max_jobs:
            raise RuntimeError("iteration exceeds the encode table capacity")
        shade = span_tiles(plan.shade)
        # the fused latent launch decodes as it shades: no decode tiles
        decode = span_tiles([] if self.fused else plan.decode)
        if max(shade[0].size, decode[0].size) > self.max_tiles:
            raise RuntimeError("iteration exceeds the tile table capacity")
        hp = h.data_ptr()
        C.memmove(hp + int(self.offs[0]), C.addressof(self.frames), C.sizeof(self.frames))
        n_sh = self._put_tiles(hp + int(self.offs[1]), plan.shade, shade)
        n_de = self._put_tiles(hp + int(self.offs[2]), plan.decode, decode)
        if jobs.size:
            C.memmove(hp + int(self.offs[3]), jobs.ctypes.data, jobs.nbytes)
        keep = []
        for aid in plan.encode:
            a = self.resident[aid]
            self.stream.wait_event(a["event"])     # already complete; orders the streams
            keep.append(a["spectral"])
            a["state"], a["spectral"] = "ready", None
        counts = np.array([n_sh, n_de, jobs.size, 0], dtype=np.int32)
        C.memmove(hp + int(self.offs[4]), counts.ctypes.data, 16)
        with torch.cuda.stream(self.stream):
            self.d_tables.copy_(h, non_blocking=True)
            ev_copy = torch.cuda.Event()
            ev_copy.record(self.stream)
            if self.graph is not None:
                self.graph.replay()
            else:
                self._launch_tables()
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.h_events[self.flip] = ev_copy
        self.flip ^= 1
        self.pending_free[id(ev)] = keep
        return ev

    _TILE_DT = np.dtype([("frame", "<i4"), ("pad", "<i4"), ("begin", "<i8"), ("end", "<i8")])
    _JOB_DT = np.dtype([("S", "<u8"), ("Z", "<u8"), ("ld_s", "<i8"), ("ld_z", "<i8"), ("begin", "<i8"),
                        ("end", "<i8")])

    def _put_tiles(self, dst: int, spans, tiles) -> int:
        """Write the tiles of `spans` (span_tiles(spans)) into the pinned
        table at address dst."""
        idx, begin, end = tiles
        arr = np.zeros(idx.size, self._TILE_DT)
        if idx.size:
            span_slot = np.array([self.reqs[sp[0]]["slot"] for sp in spans], dtype=np.int32)
            arr["frame"], arr["begin"], arr["end"] = span_slot[idx], begin, end
            C.memmove(dst, arr.ctypes.data, arr.nbytes)
        return int(idx.size)

    def poll(self, handle) -> bool:
        if handle.query():
            self.pending_free.pop(id(handle), None)
            return True
        return False

    def finish(self, req):
        if req.keep_result:
            req.result = self.reqs[req.rid]["xyz"].cpu().numpy()

    def release(self, req):
        # the slot's table entry stays as is: no tile refers to it any more
        self.reqs.pop(req.rid, None)

    def synchronize(self):
        self.stream.synchronize()

    def prewarm(self, nbytes: float):
        """Fill the caching allocator's pool of the backend's stream with one
        block of nbytes, which later frame buffers are carved from, so frames
        do not pay for first-touch device allocations."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            block = torch.empty(int(nbytes), dtype=torch.uint8, device=self.dev)
            del block


# ------------------------------------------------------------------ workload and driver

def _serving_config() -> dict:
    import synth
    return synth.config(3)


def make_requests(rate: float, count: int, n_assets: int, seed: int, t0: float = 0.0,
                  spps=None, l_range=None, resolutions=None):
    """Poisson arrivals at `rate` frames/s with resolution, spp and asset drawn
    uniformly (the serving workload's distributions; by default those of the
    serving configuration)."""
    cfg = _serving_config()
    spps = tuple(cfg["spp"]) if spps is None else spps
    l_range = tuple(cfg["path_length"]) if l_range is None else l_range
    resolutions = [tuple(r) for r in cfg["resolutions"]] if resolutions is None else resolutions
    rng = np.random.default_rng([3, 5, seed])
    t = t0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        w, h = resolutions[rng.integers(len(resolutions))]
        out.append(Request(rid=i, asset=int(rng.integers(n_assets)), width=w, height=h,
                           spp=int(rng.choice(spps)), l_min=l_range[0], l_max=l_range[1],
                           seed=10_000 + i, arrival=t))
    return out


def run_stream(sched: Scheduler, requests, time_limit: float = 120.0, idle_sleep: float = 2e-5):
    """Feed requests at their arrival times (seconds from now) and run the
    scheduler until all are done.  Returns wall seconds."""
    start = time.perf_counter()
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    for r in pending:
        r.arrival += start
    while pending or not sched.idle:
        now = time.perf_counter()
        if now - start > time_limit:
            raise TimeoutError("serving run exceeded its time limit")
        while pending and pending[0].arrival <= now:
            sched.submit(pending.popleft())
        if not sched.step(now):
            time.sleep(idle_sleep)
    return time.perf_counter() - start


def summarize(reqs, wall: float) -> dict:
    ok = [r for r in reqs if r.state == "done"]
    lat = np.array([r.latency for r in ok]) * 1e3
    first = np.array([r.latency for r in ok if r.first_use]) * 1e3
    warm = np.array([r.latency for r in ok if not r.first_use]) * 1e3
    verts = sum(r.expected_vertices for r in ok)
    pct = lambda x, q: float(np.percentile(x, q)) if x.size else None  # noqa: E731
    return {"requests": len(reqs), "completed": len(ok),
            "failed": sum(r.state == "failed" for r in reqs),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "mean_ms": float(lat.mean()) if lat.size else None,
            "first_use": {"requests": int(first.size), "p50_ms": pct(first, 50), "p99_ms": pct(first, 99)},
            "resident_asset": {"requests": int(warm.size), "p50_ms": pct(warm, 50), "p99_ms": pct(warm, 99)},
            "frames_per_s": len(ok) / wall, "path_vertices_per_s": verts / wall, "wall_s": wall}


def make_assets(n_assets: int | None = None, n: int | None = None, seed: int = 3):
    """Spectral textures in pinned host memory, the serving configuration's
    sides (512, 1024, 2048) in turn, each a Perlin-weighted blend of its own
    16 basis reflectances (weight maps of the larger sides are the 512^2 map
    repeated per texel block)."""
    import torch

    import synth
    from .layout import line_stride
    cfg = _serving_config()
    tx = cfg["texture"]
    n_assets = cfg["assets"] if n_assets is None else n_assets
    n = cfg["n"] if n is None else n
    ps = tx["perlin_side"]
    wmap = synth.perlin_weights(tx["perlin_seed"], ps)
    rng = np.random.default_rng([3, 1, seed])
    ld = line_stride(n)
    out = []
    for a in range(n_assets):
        side = tx["sides"][a % len(tx["sides"])]
        f = side // ps
        w = wmap.reshape(ps, ps, -1)
        if f > 1:
            w = np.repeat(np.repeat(w, f, axis=0), f, axis=1)
        basis = synth.reflectances(rng, n, tx["basis"]).astype(np.float32)
        tex = torch.zeros(side * side, ld, dtype=torch.float32).pin_memory()
        tex[:, :n] = torch.from_numpy(w.reshape(side * side, -1).astype(np.float32) @ basis)
        out.append(tex)
    return out


def bench_serving(device, rates=None, count: int | None = None, E=None, D=None, assets=None,
                  progress=None):
    """p50 / p99 frame latency and throughput of latent and spectral serving of
    the same request streams.  progress(str), if given, gets a line per run."""
    import torch

    import synth
    cfg = _serving_config()
    rates = tuple(cfg["rates_fps"]) if rates is None else rates
    count = cfg["requests_per_rate"] if count is None else count
    n, lt = cfg["n"], cfg["lights"]
    rng = np.random.default_rng([3, 0])
    lights = torch.from_numpy(synth.illuminant_table(rng, n, lt["planck"], lt["narrow"], *lt["narrow_sigma_nm"]))
    T = torch.from_numpy(synth.cmf_matrix(n))
    if E is None:
        E, D = (torch.from_numpy(x) for x in synth.codec_uniform(np.random.default_rng([3, 3]), cfg["k"], n))
    assets = assets if assets is not None else make_assets(cfg["assets"], n)
    out = {"rates_fps": list(rates), "requests_per_rate": count,
           "start": "each (form, rate) run starts with no asset resident"}
    for form in ("latent", "spectral"):
        res = {}
        for rate in rates:
            be = GpuBackend(assets, lights, T, E, D, form=form, device=device)
            be.prewarm(24e9)   # no run pays first-touch allocations
            reqs = make_requests(rate, count, len(assets), seed=int(rate))
            sched = Scheduler(be)  # memory budget: the device's free memory
            wall = run_stream(sched, reqs, time_limit=max(120.0, 3.0 * count / rate))
            be.synchronize()
            s = summarize(reqs, wall)
            s.update(iterations=sched.iterations, mem_budget_bytes=sched.mem_budget,
                     mem_peak_bytes=sched.mem_peak, asset_evictions=sched.evictions)
            res[str(rate)] = s
            if progress is not None:
                progress(f"serving {form} {rate} fps: {s['completed']}/{count} requests, "
                         f"p50 {s['p50_ms']:.2f} ms, p99 {s['p99_ms']:.2f} ms")
            del be, sched
            torch.cuda.empty_cache()   # the next run's stream cannot reuse this pool
        out[form] = res
    return out


def bench_saturation(device, asset, lights, T, E, D, frames: int = 8, width: int = 3840,
                     height: int = 2160, spp: int = 64, l_range=(1, 8), mem_budget: float = 150e9,
                     iter_vertices: float = 400e6, grid: int = 0, target_tiles: int = 4096,
                     max_tiles: int = 8192, forms=("latent", "spectral")) -> dict:
    """Serving at saturation: a burst of `frames` identical-shape requests
    (default 4K, 64 spp, path length 1..8) on one asset, all arriving at once,
    after a small warm-up request has brought the asset in (and encoded it).
    Reports throughput and per-frame latency for both forms.  asset: pinned
    host float32 (texels, ld) spectral texture."""
    import torch

    out = {"frames": frames, "width": width, "height": height, "spp": spp, "path_length": list(l_range),
           "mem_budget_bytes": mem_budget, "iteration_vertices": iter_vertices, "grid": grid,
           "target_tiles": target_tiles}
    for form in forms:
        be = GpuBackend([asset], lights, T, E, D, form=form, device=device, grid=grid,
                        max_tiles=max_tiles)
        be.prewarm(mem_budget)
        sched = Scheduler(be, mem_budget=mem_budget, iter_vertices=iter_vertices,
                          target_tiles=target_tiles, max_tiles=max_tiles)
        warm = Request(rid=10_000, asset=0, width=256, height=256, spp=1, l_min=1, l_max=1, seed=1)
        run_stream(sched, [warm])
        be.synchronize()
        reqs = [Request(rid=i, asset=0, width=width, height=height, spp=spp, l_min=l_range[0],
                        l_max=l_range[1], seed=20_000 + i, arrival=0.0) for i in range(frames)]
        it0 = sched.iterations
        wall = run_stream(sched, reqs, time_limit=600.0)
        be.synchronize()
        s = summarize(reqs, wall)
        s["iterations"] = sched.iterations - it0
        out[form] = s
        del be, sched
        torch.cuda.empty_cache()
    return out
