"""Benchmark of the latent (k = 6) and spectral (n = 31) light-path paths on one GPU.

Workload: 1920 x 1080 pixels, 16 samples per pixel, path length uniform in
1..4 reflectance vertices, a 1024^2 x 31 Perlin-blended spectral texture
sampled at uniform random texels, 32 lights (16 Planckian, 16 narrow-band).
All inputs are seeded synthetic data resident in HBM before timing.

A timed step is one latent frame: encode the texture and the lights with the
codec (Eq. 4), shade every path in code space with the fused B = 2 blockwise
passes and the per-pixel sample mean (Eq. 6), decode the latent image to XYZ.
`value` is path-vertices per second of that step.  The spectral form of the
same frame is timed the same way for the latent/spectral speedup, and the
CIEDE2000 of latent against spectral XYZ is reported under a codec fitted on
the GPU beforehand.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "1920x1080 px, 16 spp, path length 1-4, 1024^2 x 31 Perlin texture, 32 lights, latent k=6"
STRESS = ("3840x2160 px, 64 spp, path length 1-8, 4096^2 x 81 texture, 256 lights "
          "(75% narrow-band), latent k=9")


def codec_config() -> dict:
    """The codec-fit workload's configuration (batch, Adam, steps, loss weights)."""
    import synth
    return synth.config(2)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ CPU baseline (oracle)

_W = None


def _oracle_chunk(job):
    """Oracle latent pipeline (FP64) on a chunk of frame pixels; returns
    (path-vertices, seconds).  With `subset` the oracle is handed only the
    texture rows the chunk's records reach (texel indices renumbered into
    them), which changes no product and keeps it from converting a
    multi-gigabyte table to FP64 per chunk."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import shade as osh
    from synth import records_of_pixels
    pixels, subset = job
    w = _W
    hdr, pf, vtx = records_of_pixels(w["paths"], pixels)
    tex = w["refl"][:, :w["n"]]
    if subset:
        used, inv = np.unique(vtx[:, 0], return_inverse=True)
        vtx = vtx.copy()
        vtx[:, 0] = inv.astype(vtx.dtype)
        tex = tex[used]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        osh.render_latent_xyz(hdr, pf, vtx, w["paths"].spp, tex, w["illum"], w["E"], w["D"], w["T"])
        dt = time.perf_counter() - t0
    return int(vtx.shape[0]), dt


def cpu_baseline_small_frame(w0, reps=3):
    """The oracle on the small frame (256 x 256, 1 spp, one vertex per path)
    in full, one process: its spectral and latent (encode, shade, decode)
    pipelines, best of `reps`."""
    from oracle import shade as osh
    from synth import gen_paths
    hdr, pf, vtx = gen_paths(w0["paths"])
    spp = w0["paths"].spp
    out = {}
    for form in ("spectral", "latent"):
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            if form == "spectral":
                osh.shade_spectral(hdr, pf, vtx, spp, w0["refl"], w0["illum"], w0["T"])
            else:
                osh.render_latent_xyz(hdr, pf, vtx, spp, w0["refl"], w0["illum"], w0["E"], w0["D"], w0["T"])
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        out[f"{form}_ms"] = best * 1e3
    out.update(path_vertices=int(vtx.shape[0]), cores=1, kind="oracle",
               value=int(vtx.shape[0]) / (out["latent_ms"] * 1e-3), unit="path-vertices/s (latent)")
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def small_frame_gpu(w0, dev, reps=50):
    """The small frame (256 x 256, 1 spp, 64 materials, 8 lights, k = 6) in
    full on the GPU: the latent step (encode materials and lights, decoder
    matrix, shading with the decode) and the spectral step, HIP events over
    `reps` back-to-back steps each (launch-bound at this size)."""
    import torch
    from paper_2602_18741_amd import ops
    spec = w0["paths"]
    P = ops.gen_paths(spec.n_pixels, spec.spp, spec.l_min, spec.l_max, spec.n_tex, spec.n_illum, spec.seed,
                      device=dev)
    refl = ops.padded(torch.from_numpy(w0["refl"]).to(dev))
    illum = ops.padded(torch.from_numpy(w0["illum"]).to(dev))
    E, D, T = (torch.from_numpy(w0[x]).to(dev) for x in ("E", "D", "T"))
    k, n = E.shape
    codes = torch.empty(refl.shape[0], ops.latent_width(k), device=dev)
    lcodes = torch.empty(illum.shape[0], ops.latent_width(k), device=dev)
    M = torch.empty(3, 3 * ops.blocks(k), device=dev)
    xyz = torch.empty(spec.n_pixels, 3, device=dev)

    def latent():
        ops.encode(E, refl, n=n, out=codes)
        ops.encode(E, illum, n=n, out=lcodes)
        ops.decode_matrix(D, T, k, out=M)
        ops.shade_latent_xyz(P, codes, lcodes, M, k, out=xyz)

    def spectral():
        ops.shade_spectral(P, refl, illum, T, n, out=xyz)

    out = {"pixels": spec.n_pixels, "spp": spec.spp, "path_vertices": int(P.n_vertices)}
    for name, step in (("latent", latent), ("spectral", spectral)):
        for _ in range(5):
            step()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step()
        e1.record()
        torch.cuda.synchronize()
        out[f"{name}_step_ms"] = e0.elapsed_time(e1) / reps
    out["latent_path_vertices_per_s"] = out["path_vertices"] / (out["latent_step_ms"] * 1e-3)
    return out


def cpu_baseline(w, n_pixels=None, chunk=32768, subset=False, what="the frame"):
    """Time the oracle on a pixel sample of the frame with a pool of worker
    processes (forked before any GPU use, one BLAS thread each)."""
    import multiprocessing as mp
    import numpy as np
    global _W
    _W = w
    workers = max(1, min(16, os.cpu_count() or 1))
    if n_pixels is None:
        n_pixels = w["paths"].n_pixels
    rng = np.random.default_rng(12)
    pix = np.sort(rng.choice(w["paths"].n_pixels, n_pixels, replace=False))
    chunks = [(pix[i:i + chunk], subset) for i in range(0, n_pixels, chunk)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_chunk, chunks)
        wall = time.perf_counter() - t0
    verts = sum(r[0] for r in res)
    return {"value": verts / wall, "unit": "path-vertices/s", "cores": workers, "kind": "oracle",
            "sample": f"{n_pixels} pixels of {what} ({verts} path-vertices), FP64 numpy "
                      f"latent pipeline (encode, shade, decode) in {len(chunks)} chunks"
                      + (" (each given the texture rows its records reach)" if subset else "")
                      + f", {wall:.2f} s wall, {sum(r[1] for r in res):.1f} core-s"}


# ------------------------------------------------------------------ GPU part

TRAFFIC_JSON = os.path.join(ROOT, "profiles", "shade_latent_1080p16_traffic.json")
TRAFFIC_STRESS_JSON = os.path.join(ROOT, "profiles", "shade_stress_4k64_traffic.json")


def kernel_source_sha():
    """Digest of the sources the latent shading kernel is built from."""
    h = hashlib.sha256()
    for f in ("k_latent.hip", "shade_common.hpp", "decode_common.hpp", "hc_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2602_18741_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _counter_mean(csv_path, kernel_substr, counter, required=True):
    import csv
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(csv_path))
            if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        if required:
            raise SystemExit(f"no {counter} rows for {kernel_substr} in {csv_path}")
        return None
    return sum(vals) / len(vals)


TRAFFIC_NOTE = ("fetch/write: FETCH_SIZE and WRITE_SIZE of the kernel, each scaled by true bytes / "
                "counter of a 1 GiB device copy; they count what the L2 asks of the memory side, "
                "MALL hits included, so above the copy rate they are not HBM bytes. "
                "ea_read_bytes: L2-to-fabric read requests x their size (all 128 B here). "
                "dram_read_bytes: TCC_EA0_RDREQ_DRAM x 128 B, the requests the L2 sends towards "
                "memory; the L2 counters cannot tell a MALL hit from an HBM read.")


def record_traffic(d_fetch, d_write, d_copy_fetch, d_copy_write, d_req=None, stress=False):
    """Write the traffic record of one latent shading launch from rocprofv3
    --pmc CSVs (run_counter_collection.csv in each directory): FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) of the kernel scaled by the ratio of the
    true bytes of a 1 GiB device copy to what the same counter reads for that
    copy; with d_req also the L2-to-fabric read requests (TCC_EA0_RDREQ,
    TCC_EA0_RDREQ_128B, TCC_EA0_RDREQ_DRAM).  With `stress` the record is the
    stress frame's (its own file)."""
    csv = lambda d: os.path.join(d, "run_counter_collection.csv")  # noqa: E731
    gib_kib = float(1 << 20)
    kern = "shade_latent_kernel"
    f_scale = gib_kib / _counter_mean(csv(d_copy_fetch), "copyBuffer", "FETCH_SIZE")
    w_scale = gib_kib / _counter_mean(csv(d_copy_write), "copyBuffer", "WRITE_SIZE")
    fetch = _counter_mean(csv(d_fetch), kern, "FETCH_SIZE") * 1024 * f_scale
    write = _counter_mean(csv(d_write), kern, "WRITE_SIZE") * 1024 * w_scale
    d = {"kernel": ("shade_latent_kernel<3> (decode in the epilogue, table past the cache)" if stress
                    else "shade_latent_kernel<2> (decode in the epilogue)"),
         "workload": STRESS if stress else WORKLOAD,
         "kernel_source_sha": kernel_source_sha(), "fetch_scale": f_scale, "write_scale": w_scale,
         "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
         "fetch_plus_write_bytes_per_launch": fetch + write, "note": TRAFFIC_NOTE}
    if d_req:
        req = {c: _counter_mean(csv(d_req), kern, c, required=False)
               for c in ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_DRAM_sum")}
        d["ea_read_requests"] = req["TCC_EA0_RDREQ_sum"]
        d["ea_read_bytes"] = None if req["TCC_EA0_RDREQ_128B_sum"] is None else 128 * req["TCC_EA0_RDREQ_128B_sum"]
        d["dram_read_requests"] = req["TCC_EA0_RDREQ_DRAM_sum"]
        d["dram_read_bytes"] = None if req["TCC_EA0_RDREQ_DRAM_sum"] is None else 128 * req["TCC_EA0_RDREQ_DRAM_sum"]
    json.dump(d, open(TRAFFIC_STRESS_JSON if stress else TRAFFIC_JSON, "w"), indent=1)
    print(json.dumps(d))


def stream_bandwidth(dev, reps: int = 10) -> dict:
    """Sequential bandwidth of the device from the streaming probe
    (hc_stream_probe) over 1 GiB: copy (2 GiB moved per pass, read + write)
    and read-only, each the best of grids of 1, 2, 4 and 8 workgroups per
    CU, HIP events around `reps` back-to-back passes."""
    import torch
    from paper_2602_18741_amd import ops
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    src = torch.ones(1 << 28, device=dev)
    dst = torch.empty_like(src)
    out = {}
    for mode, moved in (("copy", 2), ("read", 1)):
        best = None
        for per_cu in (1, 2, 4, 8):
            grid = per_cu * cus
            ops.stream_probe(src, dst, mode, grid)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                ops.stream_probe(src, dst, mode, grid)
            e1.record()
            torch.cuda.synchronize()
            gbs = reps * moved * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
            if best is None or gbs > best[0]:
                best = (gbs, per_cu)
        out[f"{mode}_GBs"], out[f"{mode}_workgroups_per_cu"] = best
    del src, dst
    torch.cuda.empty_cache()
    return out


def attach_traffic(roof, traffic, kern_s):
    """Add a traffic record (or None) to a roofline entry: `traffic` is the
    counted fetch + write bytes per launch, `traffic_GBs` their rate over
    the kernel time measured in this run."""
    roof["traffic"] = None if traffic is None else traffic["fetch_plus_write_bytes_per_launch"]
    if traffic is not None:
        roof["traffic_note"] = traffic["note"]
        for key in ("fetch_bytes_per_launch", "write_bytes_per_launch", "ea_read_bytes", "dram_read_bytes"):
            roof[f"traffic_{key}"] = traffic.get(key)
        roof["traffic_GBs"] = traffic["fetch_plus_write_bytes_per_launch"] / kern_s / 1e9


def measured_traffic(stress=False):
    """Traffic record of the latent shading launch (the 1080p frame, or the
    stress frame) from the committed counter profile, if it was taken with the
    current kernel source; else None."""
    path = TRAFFIC_STRESS_JSON if stress else TRAFFIC_JSON
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None
    d.setdefault("note", TRAFFIC_NOTE)
    return d


def gather_ceiling(vtx, table, row_floats, lanes, dev, reps=3):
    """The random-gather probe (hc_gather_probe) over these records and this
    table, for unroll 1..8 and grids of 2, 4 and 8 workgroups per CU: the
    best vertex (row) rate, HIP events on the launch stream."""
    import torch
    from paper_2602_18741_amd import ops
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    nv = int(vtx.shape[0])
    best = None
    out = torch.empty(8 * cus * 256, device=dev)
    for per_cu in (2, 4, 8):
        for unroll in (1, 2, 4, 8):
            grid = per_cu * cus
            ops.gather_probe(vtx, table, row_floats, unroll, lanes, grid, out)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                ops.gather_probe(vtx, table, row_floats, unroll, lanes, grid, out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            if best is None or ms < best["ms"]:
                best = {"ms": ms, "unroll": unroll, "workgroups_per_cu": per_cu}
    best.update(rows_per_s=nv / (best["ms"] * 1e-3), rows=nv, row_bytes=4 * row_floats,
                lanes_per_row=lanes, table_bytes=int(table.numel()) * 4)
    return best


def random_records(nv, n_rows, dev, seed=7):
    """nv records with uniform random texels in [0, n_rows) and weight 1."""
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    vtx = torch.empty(nv, 2, dtype=torch.int32, device=dev)
    vtx[:, 0] = torch.randint(0, n_rows, (nv,), device=dev, generator=g, dtype=torch.int32)
    vtx[:, 1] = 0x3F800000
    return vtx


def frame_roofline(kernel, bytes_alg, kern_s, nv, ceiling, copy_gbs, limiter):
    """Roofline entry of one shading kernel: algorithmic bytes per launch over
    its time against the 8 TB/s HBM peak, and its vertex rate against the
    random-gather ceiling of the same records and table."""
    achieved = bytes_alg / kern_s / 1e9
    rate = nv / kern_s
    return {"bound": "hbm", "limiter": limiter, "kernel": kernel, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "algorithmic_bytes": bytes_alg, "kernel_ms": kern_s * 1e3, "path_vertices_per_s": rate,
            "gather_ceiling_rows_per_s": ceiling["rows_per_s"], "frac_of_gather_ceiling":
                rate / ceiling["rows_per_s"], "gather_ceiling": ceiling,
            "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs}


def stress_leg(w, args, dev, copy_gbs, cpu):
    """Config-4 frame (3840 x 2160, 64 spp, path length 1..8, 4096^2 x 81
    texture, 256 lights): both forms timed as single frames with the codec
    fitted at n = 81, k = 9, per-form roofline and gather ceiling (tables of
    1 GiB and 6.4 GB, past the 256 MB cache), CIEDE2000 of latent against
    spectral, and the oracle timed on 16,384 pixels (taken before GPU use)."""
    import numpy as np
    import torch
    import synth
    from paper_2602_18741_amd import colour, ops
    from paper_2602_18741_amd.codec_fit import CodecFit
    from paper_2602_18741_amd.layout import latent_width, line_stride
    n, k = 81, 9
    ld_z = line_stride(latent_width(k))
    spec = w["paths"]
    t0 = time.time()
    refl = torch.from_numpy(w["refl"]).to(dev)
    illum = ops.padded(torch.from_numpy(w["illum"]).to(dev))
    T = torch.from_numpy(w["T"]).to(dev)
    P = ops.gen_paths(spec.n_pixels, spec.spp, spec.l_min, spec.l_max, spec.n_tex, spec.n_illum,
                      spec.seed, device=dev)
    nv, npath, npx = P.n_vertices, spec.n_paths, spec.n_pixels
    pa, pb = synth.workloads.codec_pools(n, 1 << 18)
    pa, pb = torch.from_numpy(pa).to(dev), torch.from_numpy(pb).to(dev)
    we0, wd0 = synth.codec_init(np.random.default_rng([2, 3]), k, n)
    cc = codec_config()
    fit = CodecFit(we0, wd0, pa, pb, batch=cc["batch"], lr=cc["adam"]["lr"], seed=2, objective="eq8",
                   T=w["T"])
    fit.run(1)
    fit.capture(CODEC_STEPS_PER_GRAPH)
    loss = float(fit.run(cc["steps"] - 1))
    E, D = fit.weights()
    del pa, pb, fit
    log(f"stress frame: {npx} px, {npath} paths, {nv} path-vertices; inputs on the GPU and codec "
        f"fitted ({cc['steps']} steps, loss {loss:.4g}) in {time.time() - t0:.1f} s")
    codes = torch.empty(spec.n_tex, ld_z, device=dev)
    lcodes = torch.empty(spec.n_illum, ld_z, device=dev)
    Mdec = torch.empty(3, 3 * ops.blocks(k), device=dev)
    xyz_l = torch.empty(npx, 3, device=dev)
    xyz_s = torch.empty(npx, 3, device=dev)

    def latent_step(ev=None):
        ops.encode(E, refl, n=n, out=codes)
        ops.encode(E, illum, n=n, out=lcodes)
        ops.decode_matrix(D, T, k, out=Mdec)
        if ev:
            ev[0].record()
        ops.shade_latent_xyz(P, codes, lcodes, Mdec, k, out=xyz_l)
        if ev:
            ev[1].record()

    def spectral_step(ev=None):
        if ev:
            ev[0].record()
        ops.shade_spectral(P, refl, illum, T, n, out=xyz_s)
        if ev:
            ev[1].record()

    res = {}
    for name, step in (("latent", latent_step), ("spectral", spectral_step)):
        step()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.stress_steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for e in evs:
            step(e)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t1) / args.stress_steps
        kern = sum(a.elapsed_time(b) for a, b in evs) / args.stress_steps / 1e3
        res[name] = (wall, kern)
        log(f"stress {name}: step {wall * 1e3:.2f} ms, shade kernel {kern * 1e3:.2f} ms")
    de = colour.frame_difference(xyz_s.cpu().numpy(), xyz_l.cpu().numpy())
    log(f"stress CIEDE2000 latent vs spectral: mean {de['mean']:.3f}, p95 {de['p95']:.3f}")
    del xyz_l, xyz_s
    ceil_l = gather_ceiling(P.vtx, codes, 4 * ops.blocks(k), 1, dev, reps=2)
    ceil_s = gather_ceiling(P.vtx, refl, 4 * ((n + 3) // 4), 8, dev, reps=2)
    log(f"stress gather ceilings: codes {ceil_l['rows_per_s'] / 1e9:.1f} G rows/s, "
        f"spectra {ceil_s['rows_per_s'] / 1e9:.1f} G rows/s")
    bytes_lat = npath * 4 + nv * (8 + 4 * k) + npx * (12 + 4)
    bytes_spe = npath * 4 + nv * (8 + 4 * n) + npx * (12 + 4)
    lat = frame_roofline(f"shade_latent_kernel<{ops.blocks(k)}> (decode in the epilogue)", bytes_lat,
                         res["latent"][1], nv, ceil_l,
                         copy_gbs, "random 64-byte code rows from a 1 GiB table in HBM (one 128-byte "
                         "line each)")
    attach_traffic(lat, measured_traffic(stress=True), res["latent"][1])
    spe = frame_roofline("shade_spectral_kernel (n = 81)", bytes_spe, res["spectral"][1], nv, ceil_s, copy_gbs,
                         "random 384-byte spectral rows from a 6.4 GB table in HBM (three 128-byte "
                         "lines each)")
    out = {"workload": STRESS, "pixels": npx, "spp": spec.spp, "paths": npath, "path_vertices": nv,
           "n": n, "k": k, "codec": {"objective": "eq8", "steps": cc["steps"], "loss": loss},
           "latent": {"value": nv / res["latent"][0], "unit": "path-vertices/s",
                      "ms_per_step": res["latent"][0] * 1e3, "roofline": lat},
           "spectral": {"value": nv / res["spectral"][0], "unit": "path-vertices/s",
                        "ms_per_step": res["spectral"][0] * 1e3, "roofline": spe},
           "speedup_latent_vs_spectral": res["spectral"][0] / res["latent"][0],
           "shade_speedup_latent_vs_spectral": res["spectral"][1] / res["latent"][1],
           "ciede2000_latent_vs_spectral": de, "cpu_baseline": cpu}
    del P, refl, codes, lcodes, illum
    torch.cuda.empty_cache()
    return out


CODEC_STEPS_PER_GRAPH = 8   # fit steps (codec, upsampler) recorded in one HIP graph


def codec_only(args):
    """--codec-steps graph-replayed codec steps of each objective (n =
    args.codec_n, k = args.k, batch 65,536, pools of 2^20): the step time
    alone."""
    import numpy as np
    import torch
    import synth
    from paper_2602_18741_amd.codec_fit import CodecFit
    n, k = args.codec_n, args.k
    pa, pb = synth.workloads.codec_pools(n, 1 << 20)
    pa, pb = torch.from_numpy(pa).cuda(), torch.from_numpy(pb).cuda()
    we0, wd0 = synth.codec_init(np.random.default_rng([2, 3]), k, n)
    for objective in ("eq8", "l2"):
        fit = CodecFit(we0, wd0, pa, pb, batch=codec_config()["batch"], seed=2, objective=objective,
                       T=synth.cmf_matrix(n))
        fit.run(1)
        fit.capture(CODEC_STEPS_PER_GRAPH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = float(fit.run(args.codec_steps))
        torch.cuda.synchronize()
        log(f"codec {objective}: {(time.perf_counter() - t0) * 1e6 / args.codec_steps:.1f} us/step, "
            f"loss {loss:.4g}")


def codec_step_timing(n, k, steps, dev):
    """Graph-replayed codec fit steps (batch 65,536, pools of 2^18) of both
    objectives at one (n, k): microseconds per step."""
    import numpy as np
    import torch
    import synth
    from paper_2602_18741_amd.codec_fit import CodecFit
    pa, pb = synth.workloads.codec_pools(n, 1 << 18)
    pa, pb = torch.from_numpy(pa).to(dev), torch.from_numpy(pb).to(dev)
    we0, wd0 = synth.codec_init(np.random.default_rng([2, 3]), k, n)
    batch = codec_config()["batch"]
    out = {"n": n, "k": k, "batch": batch, "steps": steps}
    for objective in ("eq8", "l2"):
        fit = CodecFit(we0, wd0, pa, pb, batch=batch, seed=2, objective=objective, T=synth.cmf_matrix(n))
        fit.run(1)
        fit.capture(CODEC_STEPS_PER_GRAPH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fit.run(steps)
        torch.cuda.synchronize()
        out[f"{objective}_us_per_step"] = (time.perf_counter() - t0) * 1e6 / steps
    return out


def multibounce_leg(args, dev, n, k, T, codecs):
    """Multi-bounce chains (Eq. 10): both forms on the codec-fit configuration's held-out chains
    of 3 bounces for each fitted codec; GPU time of one evaluation (encode,
    both shades, decode) and the CIE94 report per bounce."""
    import torch
    import synth
    from paper_2602_18741_amd import multibounce, ops
    mb = codec_config()["multibounce"]
    chains, bounces = mb["chains"], mb["bounces"]
    r, l = synth.workloads.bounce_chains(n, chains, bounces)
    r = ops.padded(torch.from_numpy(r).to(dev))
    l = ops.padded(torch.from_numpy(l).to(dev))
    paths = multibounce.chain_paths(chains, bounces, dev)
    out = {"chains": chains, "bounces": bounces, "white": "equal-energy at the light's Y",
           "cie94": {}}
    for name, ((E_, D_), _) in codecs.items():
        res = multibounce.chain_xyz(E_, D_, T, r, l, k, n, bounces, paths=paths)
        out["cie94"][name] = multibounce.cie94_report(*res)
    (E_, D_), _ = codecs["eq8"]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    reps = 10
    for _ in range(reps):
        multibounce.chain_xyz(E_, D_, T, r, l, k, n, bounces, paths=paths)
    e1.record()
    torch.cuda.synchronize()
    out["ms_per_evaluation"] = e0.elapsed_time(e1) / reps
    log("multi-bounce CIE94 mean per bounce: " + "; ".join(
        f"{name} " + ", ".join(f"{b['mean']:.3f}" for b in rep) for name, rep in out["cie94"].items())
        + f"; {out['ms_per_evaluation']:.3f} ms per evaluation of {chains} chains")
    return out


UP_SIDE = 4096           # RGB texture side for the upsampling throughput
MFMA_F16_PEAK_TFS = 2500.0
MFMA_F32_PEAK_TFS = 157.3


ENGINE_CLOCK_GHZ = 2.4     # peak engine clock
SIMDS = 256 * 4            # 256 compute units of 4 SIMDs


def alu_issue_rates(dev, grid: int = 2048) -> dict:
    """Cycles per wavefront instruction per SIMD, at the peak engine clock,
    of each kind of the issue-rate probe (hc_alu_probe) with 8 wavefronts per
    SIMD: the cost of the activation's exponential and reciprocal, in fp32
    and fp16, against a multiply-add."""
    import torch
    from paper_2602_18741_amd import ops
    out = torch.empty(grid * 256, dtype=torch.float32, device=dev)
    instr = grid * 4 * ops.ALU_PROBE_CHAINS * ops.ALU_PROBE_ITERS
    rates = {}
    for op in ops.ALU_PROBE_OPS:
        ops.alu_probe(op, out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            ops.alu_probe(op, out)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        rates[op] = sec * ENGINE_CLOCK_GHZ * 1e9 * SIMDS / instr
    return rates


def upsample_throughput(net: dict, k: int, dev) -> dict:
    """The upsampling network on a 4096^2 RGB texture in both precisions
    (HIP events over 10 back-to-back launches), with the issue rates of the
    fp16 kernel's instructions (hc_alu_probe)."""
    import torch
    from paper_2602_18741_amd import ops
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    rgb_big = torch.rand(UP_SIDE * UP_SIDE, 4, device=dev, generator=g)
    out = torch.empty(UP_SIDE * UP_SIDE, ops.latent_width(k), device=dev)
    flop = 2.0 * (3 * 128 + 128 * 128 + 128 * k) * rgb_big.shape[0]
    timing = {}
    for prec, peak in (("f16", MFMA_F16_PEAK_TFS), ("f32", MFMA_F32_PEAK_TFS)):
        for _ in range(2):
            ops.upsample(net, rgb_big, k, precision=prec, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            ops.upsample(net, rgb_big, k, precision=prec, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tfs = flop / (ms * 1e-3) / 1e12
        timing[prec] = {"ms": ms, "texels_per_s": rgb_big.shape[0] / (ms * 1e-3), "TFLOP_s": tfs,
                        "mfma_peak_TFLOP_s": peak, "frac": tfs / peak}
    log("upsampling 4096^2 texels: " + ", ".join(
        f"{p} {v['ms']:.3f} ms ({v['TFLOP_s']:.0f} TFLOP/s)" for p, v in timing.items()))
    # the f16 kernel's time goes mostly to its vector instructions (an
    # exponential and a reciprocal per activation), not the matrix cores
    timing["f16"]["alu_issue_cycles"] = alu_issue_rates(dev)
    log("issue cycles per wavefront instruction: " + ", ".join(
        f"{op} {c:.2f}" for op, c in timing["f16"]["alu_issue_cycles"].items()))
    return timing


def upsample_leg(args, dev, n, k, T, E, D, refl, illum, P, xyz_s, codes, lcodes, zimg, xyz_l):
    """RGB-to-latent upsampling (Sec. 5): fit the network on the GPU against
    the frozen codec (reflectance pool, AdamW), time it on a 4096^2 RGB
    texture in both precisions, and shade the frame with the upsampled
    texture codes (spectral lights encoded as usual)."""
    import numpy as np
    import torch
    import synth
    from paper_2602_18741_amd import colour, ops
    from paper_2602_18741_amd.upsample_fit import UpsampleFit, training_pairs
    Tn = T.cpu().double().numpy()
    Dn = D.cpu().double().numpy()
    M = torch.from_numpy((Tn @ Dn).astype(np.float32)).to(dev)      # XYZ of a code
    white = Tn.sum(axis=1)                                            # XYZ of the unit spectrum
    pool, _ = synth.workloads.codec_pools(n, 1 << 18)
    pool = ops.padded(torch.from_numpy(pool).to(dev))
    rgb_pool, z_pool = training_pairs(E, T, pool, n)
    fit = UpsampleFit(rgb_pool, z_pool, M, white, k, batch=1024, seed=4)
    first = float(fit.run(1))
    fit.capture(CODEC_STEPS_PER_GRAPH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = float(fit.run(args.upsample_steps - 1))
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) * 1e6 / max(1, args.upsample_steps - 1)
    net = fit.net()
    log(f"upsampler fit: loss {first:.4g} -> {loss:.4g} in {fit.steps_done} steps, {us:.1f} us/step")

    # held-out reflectances: colour error of upsampled codes against the truth and the codec
    test, _ = synth.workloads.bounce_chains(n, 1 << 16, 1)
    test = ops.padded(torch.from_numpy(test).to(dev))
    rgb_t, z_t = training_pairs(E, T, test, n)
    z_up = ops.upsample(net, rgb_t, k, precision="f16")
    xyz_up = ops.decode_xyz(D, T, z_up, k).cpu().double().numpy()
    xyz_codec = ops.decode_xyz(D, T, z_t, k).cpu().double().numpy()
    xyz_true = test[:, :n].cpu().double().numpy() @ Tn.T
    lab = lambda x: colour.xyz_to_lab(x, white)  # noqa: E731
    de = lambda a, b: float(np.linalg.norm(lab(a) - lab(b), axis=1).mean())  # noqa: E731
    quality = {"test_reflectances": int(test.shape[0]),
               "de76_upsampled_vs_spectral": de(xyz_true, xyz_up),
               "de76_upsampled_vs_codec": de(xyz_codec, xyz_up),
               "de76_codec_vs_spectral": de(xyz_true, xyz_codec)}

    timing = upsample_throughput(net, k, dev)

    # the frame shaded with upsampled texture codes
    rgb_tex, _ = training_pairs(E, T, refl, n)
    ops.upsample(net, rgb_tex, k, precision="f16", out=codes)
    ops.encode(E, illum, n=n, out=lcodes)
    ops.shade_latent(P, codes, lcodes, k, out=zimg)
    ops.decode_xyz(D, T, zimg, k, out=xyz_l)
    frame = colour.frame_difference(xyz_s.cpu().numpy(), xyz_l.cpu().numpy())
    log(f"frame with upsampled texture codes: CIEDE2000 mean {frame['mean']:.3f}, p95 {frame['p95']:.3f}")
    return {"fit": {"steps": fit.steps_done, "batch": 1024, "lr": 2e-3, "first_loss": first,
                    "final_loss": loss, "us_per_step": us},
            "colour": quality, "throughput_4096sq": timing,
            "ciede2000_frame_upsampled_texture_vs_spectral": frame}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--k", type=int, default=6)
    ap.add_argument("--config", type=int, choices=[1, 4], default=1,
                    help="the main frame's workload configuration (synth/configs/cfg<N>.json): 1 the "
                         "1920x1080 frame, 4 the 3840x2160 stress frame (as --stress)")
    ap.add_argument("--codec-steps", type=int, default=None,
                    help="Adam steps of the codec fit (default: the codec-fit configuration's; the "
                         "step time and the loss after 2,000 steps, the fitting recipe's length, are "
                         "reported as well)")
    ap.add_argument("--codec-n", type=int, default=31, choices=[31, 81],
                    help="samples per spectrum of the --only codec run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-upsample", action="store_true")
    ap.add_argument("--saturation-frames", type=int, default=8,
                    help="frames in the burst of the stress workload's serving run")
    ap.add_argument("--upsample-steps", type=int, default=5000,
                    help="AdamW steps of the upsampling network's fit")
    ap.add_argument("--serve-count", type=int, default=None,
                    help="requests per arrival rate in the serving measurement (default: the "
                         "serving configuration's)")
    ap.add_argument("--no-stress", action="store_true",
                    help="leave out the 3840x2160 / 64 spp / n=81 / k=9 single-frame leg")
    ap.add_argument("--stress-steps", type=int, default=3,
                    help="timed frames per form in the stress leg (one untimed first)")
    ap.add_argument("--record-traffic", nargs="+", metavar="DIR",
                    help="rocprofv3 --pmc output directories: fetch, write, copy-fetch, copy-write "
                         "[, requests] -> traffic record of the latent shading kernel")
    ap.add_argument("--stress", action="store_true",
                    help="the 4K / 64 spp / n=81 / k=9 stress frame instead of the default frame")
    ap.add_argument("--only", choices=["latent", "spectral", "copy", "codec", "gather", "upsample"],
                    help="run only the timed steps of one form (or a 1 GiB device copy, or "
                         "--codec-steps graph-replayed codec steps of each objective, or the "
                         "random-gather probe over the frame's records and code table, or the "
                         "upsampling network's 4096^2 launches with random-init weights and the "
                         "issue-rate probe), for profilers; prints no JSON")
    args = ap.parse_args()
    import synth
    if args.codec_steps is None:
        args.codec_steps = synth.config(2)["steps"]
    if args.serve_count is None:
        args.serve_count = synth.config(3)["requests_per_rate"]
    if args.config == 4:
        args.stress = True
    if args.record_traffic:
        record_traffic(*args.record_traffic, stress=args.stress)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the shading path has no multi-GPU mode "
              "(frames would shard by pixel range with no exchange step).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import synth

    if args.only == "codec":
        codec_only(args)
        return
    if args.only == "upsample":
        import torch
        from paper_2602_18741_amd import ops
        from paper_2602_18741_amd.upsample_fit import default_init
        params = torch.from_numpy(default_init(args.k, 0)).to("cuda:0")
        net = {name: v.contiguous() for name, v in ops.unpack_mlp(params, args.k).items()}
        upsample_throughput(net, args.k, torch.device("cuda:0"))
        return
    if args.only == "copy":
        import torch
        x = torch.ones(1 << 28, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(args.warmup + args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copied 1 GiB", args.warmup + args.steps, "times")
        return

    from paper_2602_18741_amd.layout import latent_width, line_stride
    stress = args.stress
    wid, k, n = (4, 9, 81) if stress else (1, args.k, 31)
    # row strides that keep every texel row inside as few 128-byte lines as
    # its length allows: 31 samples -> 32 floats, 81 -> 96 (3 lines); codes
    # k = 6 -> 8 floats, k = 9 -> 16 (64 B)
    ld_tex = line_stride(n)
    ld_z = line_stride(latent_width(k))
    t_setup = time.time()
    w = synth.workload(wid, k=k, ld_tex=ld_tex)
    spec = w["paths"]
    log(f"inputs generated in {time.time() - t_setup:.1f} s")
    cpu = None if (args.no_cpu or args.only or stress) else cpu_baseline(w)
    if cpu:
        log("cpu baseline:", cpu["sample"])
    w0 = synth.workload(0) if not (args.only or stress) else None
    cpu0 = None if (w0 is None or args.no_cpu) else cpu_baseline_small_frame(w0)
    if cpu0:
        log(f"cpu baseline, small frame in full: spectral {cpu0['spectral_ms']:.1f} ms, latent "
            f"{cpu0['latent_ms']:.1f} ms ({cpu0['path_vertices']} path-vertices, one process)")
    w4 = cpu4 = None
    if not (args.only or stress or args.no_stress):
        t_setup = time.time()
        w4 = synth.workload(4, ld_tex=line_stride(81))
        log(f"stress inputs generated in {time.time() - t_setup:.1f} s")
        if not args.no_cpu:
            cpu4 = cpu_baseline(w4, n_pixels=16384, chunk=1024, subset=True,
                                what="the 3840x2160, 64 spp frame")
            log("stress cpu baseline:", cpu4["sample"])

    import torch
    from paper_2602_18741_amd import colour, ops
    from paper_2602_18741_amd.codec_fit import CodecFit

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    refl = torch.from_numpy(w["refl"]).to(dev)
    del w["refl"]
    illum = ops.padded(torch.from_numpy(w["illum"]).to(dev))
    T = torch.from_numpy(w["T"]).to(dev)
    P = ops.gen_paths(spec.n_pixels, spec.spp, spec.l_min, spec.l_max, spec.n_tex, spec.n_illum,
                      spec.seed, device=dev)
    bad = ops.check_paths(P, spec.n_tex, spec.n_illum)
    assert int(bad.sum()) == 0, "generated records failed the check"
    nv, npath, npx = P.n_vertices, spec.n_paths, spec.n_pixels
    log(f"frame: {npx} px, {npath} paths, {nv} path-vertices")

    # ---- codec fits on the GPU (reflectance / light pools, Adam, graph replay):
    # the four-term loss of Eq. 8 (the codec the frames use) and the two-term
    # squared error, for comparison
    pa, pb = synth.workloads.codec_pools(n, 1 << 20 if not args.only else 1 << 16)
    pa, pb = torch.from_numpy(pa).to(dev), torch.from_numpy(pb).to(dev)
    we0, wd0 = synth.codec_init(np.random.default_rng([2, 3]), k, n)
    codec_steps = 1 if args.only else args.codec_steps

    def fit_codec(objective):
        cc = codec_config()
        fit = CodecFit(we0, wd0, pa, pb, batch=cc["batch"], lam=cc["lambda"], beta=cc["softplus_beta"],
                       lr=cc["adam"]["lr"], seed=2, objective=objective, T=w["T"])
        recipe_steps = min(2000, codec_steps)
        fit.run(1)
        fit.capture(CODEC_STEPS_PER_GRAPH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss_recipe = float(fit.run(recipe_steps - 1))
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) * 1e6 / max(1, recipe_steps - 1)
        loss = float(fit.run(codec_steps - recipe_steps))
        log(f"codec fit ({objective}): loss {loss_recipe:.4g} after {recipe_steps} steps, "
            f"{loss:.4g} after {fit.steps_done}; {us:.1f} us/step")
        info = {"objective": objective, "steps": fit.steps_done, "batch": cc["batch"], "lr": cc["adam"]["lr"],
                "final_loss": loss, "loss_after_2000_steps": loss_recipe, "us_per_step": us}
        return fit.weights(), info

    codecs = {"eq8": fit_codec("eq8")}
    if not args.only:
        codecs["l2"] = fit_codec("l2")
    (E, D), _ = codecs["eq8"]
    del pa, pb
    # the codec step at the 380-780 nm grid (n = 81) with nine channels
    codec81 = None
    if not args.only and not stress and args.codec_steps >= 2000:
        codec81 = codec_step_timing(81, 9, 2000, dev)
        log(f"codec step n = 81, k = 9: eq8 {codec81['eq8_us_per_step']:.1f} us, "
            f"l2 {codec81['l2_us_per_step']:.1f} us")

    codes = torch.empty(spec.n_tex, ld_z, device=dev)
    lcodes = torch.empty(spec.n_illum, ld_z, device=dev)
    zimg = torch.zeros(npx, ops.latent_width(k), device=dev)
    Mdec = torch.empty(3, 3 * ops.blocks(k), device=dev)
    xyz_l = torch.empty(npx, 3, device=dev)
    xyz_s = torch.empty(npx, 3, device=dev)

    # one frame: encode the texture and the lights, form the decoder matrix
    # M = T D, shade all B passes with the per-pixel decode in the epilogue
    def latent_step(ev=None):
        ops.encode(E, refl, n=n, out=codes)
        ops.encode(E, illum, n=n, out=lcodes)
        ops.decode_matrix(D, T, k, out=Mdec)
        if ev:
            ev[0].record()
        ops.shade_latent_xyz(P, codes, lcodes, Mdec, k, out=xyz_l)
        if ev:
            ev[1].record()

    def spectral_step(ev=None):
        if ev:
            ev[0].record()
        ops.shade_spectral(P, refl, illum, T, n, out=xyz_s)
        if ev:
            ev[1].record()

    def timed(step):
        for _ in range(args.warmup):
            step()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in evs:
            step(e)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        kern = sum(a.elapsed_time(b) for a, b in evs) / args.steps / 1e3
        return wall, kern

    if args.only == "gather":
        # the sweep of gather_ceiling, then its best issue shape steps times
        latent_step()
        best = gather_ceiling(P.vtx, codes, 4 * ops.blocks(k), 1, dev)
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        for _ in range(args.warmup + args.steps):
            ops.gather_probe(P.vtx, codes, 4 * ops.blocks(k), best["unroll"], 1, best["workgroups_per_cu"] * cus)
        torch.cuda.synchronize()
        log(f"gather probe: best unroll {best['unroll']}, {best['workgroups_per_cu']} workgroups per CU, "
            f"{best['rows_per_s'] / 1e9:.1f} G rows/s; {args.warmup + args.steps} more launches over {nv} records")
        return
    if args.only:
        wall, kern = timed(latent_step if args.only == "latent" else spectral_step)
        log(f"{args.only}: step {wall * 1e3:.3f} ms, shade kernel {kern * 1e3:.3f} ms")
        return
    lat_wall, lat_kern = timed(latent_step)
    spe_wall, spe_kern = timed(spectral_step)
    log(f"latent step {lat_wall * 1e3:.3f} ms (shade {lat_kern * 1e3:.3f} ms); "
        f"spectral step {spe_wall * 1e3:.3f} ms")
    small = None
    if w0 is not None:
        small = small_frame_gpu(w0, dev)
        small["workload"] = "256x256 px, 1 spp, path length 1, 64 materials, 8 lights, latent k=6 vs n=31"
        small["cpu_baseline"] = cpu0
        log(f"small frame in full: latent step {small['latent_step_ms'] * 1e3:.1f} us, spectral "
            f"{small['spectral_step_ms'] * 1e3:.1f} us ({small['path_vertices']} path-vertices)")

    stream = stream_bandwidth(dev)
    copy_gbs = stream["copy_GBs"]
    log(f"streaming probe: copy {copy_gbs:.0f} GB/s (read + write), read {stream['read_GBs']:.0f} GB/s")

    # the streaming kernels against the streaming probe's read bandwidth: the
    # texture encode timed inside the step (4n + 4k algorithmic bytes per
    # texel), and the decode of a latent image to XYZ as its own launch (4k +
    # 12 per pixel; the step decodes in the shading kernel's epilogue, and its
    # XYZ must equal this launch's bit for bit)
    def streaming_kernels(reps=10):
        ops.shade_latent(P, codes, lcodes, k, out=zimg)
        xyz_d = torch.empty_like(xyz_l)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
        for e in evs:
            e[0].record()
            ops.encode(E, refl, n=n, out=codes)
            e[1].record()
            ops.encode(E, illum, n=n, out=lcodes)
            ops.decode_matrix(D, T, k, out=Mdec)
            ops.shade_latent_xyz(P, codes, lcodes, Mdec, k, out=xyz_l)
            e[2].record()
            ops.decode_xyz(D, T, zimg, k, out=xyz_d)
            e[3].record()
        torch.cuda.synchronize()
        out = {}
        for name, (i, j), nbytes in (("encode_texture", (0, 1), spec.n_tex * (4 * n + 4 * k)),
                                     ("decode_xyz", (2, 3), npx * (4 * k + 12))):
            sec = sum(e[i].elapsed_time(e[j]) for e in evs) / reps / 1e3
            gbs = nbytes / sec / 1e9
            out[name] = {"us": sec * 1e6, "algorithmic_bytes": nbytes, "GBs": gbs,
                         "frac_of_stream_read": gbs / stream["read_GBs"]}
        out["decode_xyz"]["in_step"] = False
        out["fused_decode_equals_decode_launch"] = bool(torch.equal(xyz_l, xyz_d))
        return out

    streaming = streaming_kernels()
    log("streaming kernels: " + ", ".join(
        f"{key} {v['us']:.1f} us ({v['GBs']:.0f} GB/s, {v['frac_of_stream_read']:.2f} of the read probe)"
        for key, v in streaming.items() if isinstance(v, dict))
        + f"; fused decode equals the decode launch: {streaming['fused_decode_equals_decode_launch']}")
    bytes_lat = npath * 4 + nv * (8 + 4 * k) + npx * (12 + 4)
    bytes_spe = npath * 4 + nv * (8 + 4 * n) + npx * (12 + 4)
    traffic = measured_traffic(stress=stress)

    # the random-gather ceiling of the frame's records: over the code table
    # and the spectral table the kernels read, and over a 1 GiB table of
    # 32-byte rows (past the 256 MB cache)
    ceil_lat = gather_ceiling(P.vtx, codes, 4 * ops.blocks(k), 1, dev)
    ceil_spe = gather_ceiling(P.vtx, refl, 4 * ((n + 3) // 4), 1 if n <= 16 else 8, dev)
    big = torch.rand(1 << 25, 8, device=dev)
    recs = random_records(nv, big.shape[0], dev)
    ceil_1g = gather_ceiling(recs, big, 8, 1, dev)
    del big, recs
    torch.cuda.empty_cache()
    log(f"gather ceilings: code table {ceil_lat['rows_per_s'] / 1e9:.1f} G rows/s, spectral table "
        f"{ceil_spe['rows_per_s'] / 1e9:.1f} G rows/s, 1 GiB table of 32-byte rows "
        f"{ceil_1g['rows_per_s'] / 1e9:.1f} G rows/s")
    tbl_mb = codes.numel() * 4 / 2 ** 20
    roof = frame_roofline(f"shade_latent_kernel<{ops.blocks(k)}> (decode in the epilogue)", bytes_lat,
                          lat_kern, nv, ceil_lat,
                          copy_gbs, f"random {4 * ops.blocks(k) * 4}-byte code rows from a "
                          f"{tbl_mb:.0f} MiB table" + (" resident in the 256 MB MALL" if tbl_mb < 256
                                                        else " in HBM") + " (one 128-byte line each)")
    attach_traffic(roof, traffic, lat_kern)
    roof["gather_ceiling_1GiB_rows_per_s"] = ceil_1g["rows_per_s"]
    roof["gather_ceiling_1GiB"] = ceil_1g
    roof_spe = frame_roofline("shade_spectral_kernel", bytes_spe, spe_kern, nv, ceil_spe, copy_gbs,
                              "random spectral rows from the texture (one 128-byte line per row at n = 31)")

    de = colour.frame_difference(xyz_s.cpu().numpy(), xyz_l.cpu().numpy())
    log(f"CIEDE2000 latent (Eq. 8 codec) vs spectral: mean {de['mean']:.3f}, p95 {de['p95']:.3f}")
    E2, D2 = codecs["l2"][0]
    ops.encode(E2, refl, n=n, out=codes)
    ops.encode(E2, illum, n=n, out=lcodes)
    ops.shade_latent(P, codes, lcodes, k, out=zimg)
    ops.decode_xyz(D2, T, zimg, k, out=xyz_l)
    de_l2 = colour.frame_difference(xyz_s.cpu().numpy(), xyz_l.cpu().numpy())
    log(f"CIEDE2000 latent (two-term codec) vs spectral: mean {de_l2['mean']:.3f}, "
        f"p95 {de_l2['p95']:.3f}")
    bounce = multibounce_leg(args, dev, n, k, T, codecs)
    up = None
    if not args.no_upsample:
        up = upsample_leg(args, dev, n, k, T, E, D, refl, illum, P, xyz_s, codes, lcodes, zimg, xyz_l)

    stress_out = None
    if w4 is not None:
        del P, zimg
        torch.cuda.empty_cache()
        t0 = time.time()
        stress_out = stress_leg(w4, args, dev, copy_gbs, cpu4)
        del w4
        log(f"stress leg measured in {time.time() - t0:.1f} s")

    serving = None
    if stress and not args.no_serve:
        from paper_2602_18741_amd.serve import bench_saturation
        host_tex = refl.cpu().pin_memory()
        del P, zimg, codes, refl
        torch.cuda.empty_cache()
        t0 = time.time()
        serving = bench_saturation(dev, host_tex, torch.from_numpy(w["illum"]), T.cpu(), E.cpu(), D.cpu(),
                                   frames=args.saturation_frames)
        log(f"serving at saturation measured in {time.time() - t0:.1f} s: " + ", ".join(
            f"{form} {v['frames_per_s']:.2f} frames/s ({v['path_vertices_per_s'] / 1e9:.1f} G path-vertices/s), "
            f"p50 {v['p50_ms']:.0f} ms, max {v['p99_ms']:.0f} ms" for form in ("latent", "spectral")
            for v in [serving[form]]))
    if not (args.no_serve or stress):
        from paper_2602_18741_amd.serve import bench_serving
        if stress_out is None:
            del P, zimg
        torch.cuda.empty_cache()
        t0 = time.time()
        serving = bench_serving(dev, count=args.serve_count, E=E.cpu(), D=D.cpu(), progress=log)
        log(f"serving measured in {time.time() - t0:.1f} s: " + ", ".join(
            f"{form} {r} fps p50 {v['p50_ms']:.2f} p99 {v['p99_ms']:.2f} ms"
            for form in ("latent", "spectral") for r, v in serving[form].items()))

    out = {
        "metric": "path-vertices/s latent k=6 vs spectral n=31; HBM GB/s; p99 frame ms",
        "note": "stress workload: latent k=9 vs spectral n=81" if stress else None,
        "value": nv / lat_wall,
        "unit": "path-vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": lat_wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": STRESS if stress else WORKLOAD, "pixels": npx, "spp": spec.spp,
                   "paths": npath,
                   "path_vertices": nv, "k": k, "n": n, "texels": spec.n_tex,
                   "lights": spec.n_illum, "step": "encode texture+lights, shade latent, decode"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "stream_probe": stream,
        "streaming_kernels": streaming,
        "spectral": {"value": nv / spe_wall, "unit": "path-vertices/s", "ms_per_step": spe_wall * 1e3,
                     "kernel_ms": spe_kern * 1e3, "achieved_GBs": bytes_spe / spe_kern / 1e9,
                     "algorithmic_bytes": bytes_spe, "roofline": roof_spe},
        "speedup_latent_vs_spectral": spe_wall / lat_wall,
        "shade_speedup_latent_vs_spectral": spe_kern / lat_kern,
        "ciede2000_latent_vs_spectral": de,
        "ciede2000_latent_vs_spectral_two_term_codec": de_l2,
        "codec_fit": {name: info for name, (_, info) in codecs.items()},
        "codec_step_n81_k9": codec81,
        "multibounce": bounce,
        "upsample": up,
        "stress": stress_out,
        "small_frame": small,
        "serving": serving,
        "env": {"device": torch.cuda.get_device_name(dev),
                "arch": getattr(torch.cuda.get_device_properties(dev), "gcnArchName", None),
                "hip": torch.version.hip,
                "torch": torch.__version__, "host_cores": os.cpu_count(), "host_cpu": cpu_model(),
                "seeds": {"paths": spec.seed, "texture": "perlin 1001 / 4001 (workloads 1 / 4)",
                          "codec_init": [2, 3]},
                "row_strides_floats": {"spectral": ld_tex, "codes": ld_z}},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
