"""Benchmark: Voronoi cell crossings per second on one MI355X.

Workload (default): the 10^6-site flared-disc grid (99% of sites from
rho ~ (R/R0)^-1 exp(-(pi/4)(z/h)^2), h = 0.125 R0 (R/R0)^1.125, R in
[1, 1000] AU, 1% uniform in the box +-1000 AU) with 8x10^6 rays, half from
the central point source and half from random sites, in mixed-precision
mode (FP32 plane tests, FP64 re-decision of close calls, FP64 winner).

A step is one pass of the whole path over the batch with inputs resident in
HBM: the coherent ray order (vor_order_rays), then vor_trace: start-cell
location, the traversal, the per-ray outputs and every segment (cell,
length) written to its stride window or, past it, to the ray's chain of
spill chunks. The grid is built once, outside the timed region (set-up, as
in the method). value = segments emitted per step / seconds per step.

roofline.traffic is the trace kernel's HBM traffic per launch from the
committed hardware-counter summary (profiles/), reported only while the
kernel sources still hash to the value recorded there (else null).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
                    [--workload flared_disc|exp_disc|clumpy|uniform_cube|flared_disc_transport|serving|
                                serving_precision|grid_quality]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Voronoi cell crossings/sec per GPU at stated accuracy; p50/p99 batch latency"
HBM_PEAK_GBS = 8000.0

# The sources the trace kernel is compiled from: a traffic figure measured
# on another version of them is not reported.
KERNEL_SOURCES = ("paper_1310_1854_amd/csrc/trace.hip", "paper_1310_1854_amd/csrc/trace_core.h",
                  "paper_1310_1854_amd/csrc/locate_core.h",
                  "paper_1310_1854_amd/csrc/vrt_internal.h", "include/voronoi_rt.h",
                  "paper_1310_1854_amd/build_lib.py")
# Counter summaries of the trace kernel per workload (profiles/).
TRAFFIC_SUMMARIES = {"flared_disc": "profiles/k_trace_flared_disc_1e6_mixed_traffic.md",
                     "exp_disc": "profiles/k_trace_exp_disc_1e5_mixed_traffic.md",
                     "clumpy": "profiles/k_trace_clumpy_4e6_mixed_traffic.md",
                     "flared_disc_transport": "profiles/k_trace_flared_disc_1e6_transport_traffic.md"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# Record layout of the benchmark grids ("auto", "fp32", "compact"; --records).
RECORDS = "auto"


def build_grid(vrt, w):
    """The grid as the benchmark builds it (set-up, outside the timed steps):
    the neighbour table and the paper's block lists (Sect. 2.3), which the
    start-cell pass of each trace uses, and the workload's density field
    bound to it (vor_grid_bind_density), which the steps read."""
    import torch
    grid = vrt.build_grid(w.sites, w.box, block_lists=True, records=RECORDS)
    grid.bind_density(torch.as_tensor(w.density, dtype=torch.float64, device="cuda").contiguous())
    return grid


def measured_traffic(workload: str):
    """(bytes per launch, summary path, L2 hit rate) of the trace kernel from
    the counter summary, or (None, reason, None) when there is none for this
    workload or the kernel sources have changed since it was taken."""
    traffic, src, fields = _traffic_fields(workload)
    hit = None
    if traffic is not None and "l2_hit_rate" in fields:
        try:
            hit = float(fields["l2_hit_rate"])
        except ValueError:
            pass
    return traffic, src, hit


def _traffic_fields(workload: str):
    rel = TRAFFIC_SUMMARIES.get(workload)
    path = os.path.join(ROOT, rel) if rel else None
    if not path or not os.path.exists(path):
        return None, "no counter summary", {}
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("workload") != workload:
        return None, "counter summary is for another workload", fields
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None, "kernel sources changed since the counters were taken", fields
    try:
        return float(fields["traffic_bytes_per_launch"]), rel, fields
    except (KeyError, ValueError):
        return None, "counter summary lacks traffic_bytes_per_launch", fields

# Launch configuration per workload: mode, segment window per ray, spill
# chunks (of 64 segments) per ray, coherent ray order, persistent kernel.
WORKLOADS = {
    "flared_disc": dict(cfg=2, mode="mixed", stride=128, spill_chunks_per_ray=0.5, ordered=True, persistent=True,
                        cpu_rays=1000),
    "exp_disc": dict(cfg=1, mode="mixed", stride=128, spill_chunks_per_ray=0.25, ordered=True, persistent=True,
                     cpu_rays=600, cpu_rays_configs=600),
    "clumpy": dict(cfg=3, mode="mixed", stride=128, spill_chunks_per_ray=1.0, ordered=True, persistent=True,
                   cpu_rays=60, cpu_rays_configs=60),
    "uniform_cube": dict(cfg=0, mode="fp64", stride=64, spill_chunks_per_ray=0.25, ordered=True, cpu_rays=10000,
                         cpu_rays_configs=10000),
    # the same disc with transport: each ray stops where tau reaches -ln u (seeded u), and both per-cell
    # tallies are deposited; kappa = 1e-3 puts the mean optical depth of the full paths near 0.9
    "flared_disc_transport": dict(cfg=2, mode="mixed", stride=128, spill_chunks_per_ray=0.5, ordered=True,
                                  persistent=True, cpu_rays=240, transport=True, kappa=1e-3),
}


def algorithmic_bytes(c: np.ndarray, n_rays: int, mode: str, transport: bool = False) -> float:
    """Bytes the method must move for one launch, from the kernel counters
    c = [segments, fallbacks, fp64 re-decisions, steps, records, ...].
    Per step: the row range (8 B) and, per neighbour record read, its index
    and site (4 + 24 B in FP64; 4 + 12 B FP32 offset in mixed mode, plus the
    winner's FP64 site, 24 B, and the FP64 records of re-decided steps). The
    figure belongs to the method, not to a layout: grids with compact 8-byte
    records are charged the same.
    Per segment: the cell density (8 B) and the output (4 B cell + 8 B
    length). Per ray: origin and direction (48 B), tau, count and status
    (13 B). With transport, per segment two tally updates (read and write
    8 B each) and per ray tau_stop, the interaction cell and distance (20 B)."""
    seg, redo, steps, recs = float(c[0]), float(c[2]), float(c[3]), float(c[4])
    per_step_recs = recs / max(steps, 1.0)
    b = 8.0 * steps + 20.0 * seg + 61.0 * n_rays
    if transport:
        b += 32.0 * seg + 20.0 * n_rays
    if mode == "fp64":
        b += 28.0 * recs
    else:
        b += 16.0 * recs + 24.0 * steps + 28.0 * redo * per_step_recs
    return b


def make_buffers(vrt, N, spec, torch, chunks=None):
    chunks = int(N * spec["spill_chunks_per_ray"]) + 1 if chunks is None else int(chunks)
    b = vrt.TraceBuffers(N, seg_stride=spec["stride"], spill_chunks=chunks, ordered=spec.get("ordered", False),
                         stops=spec.get("transport", False))
    b.transport = None
    return b


def add_transport(bufs, spec, torch, M, seed=20131854 + 77):
    """Transport inputs and outputs of a workload with transport: tau_stop =
    -ln u per ray (seeded), zeroed per-cell tallies."""
    if not spec.get("transport"):
        return
    g = torch.Generator(device="cpu").manual_seed(seed)
    u = torch.rand(bufs.N, generator=g, dtype=torch.float64)
    bufs.transport = dict(tau_stop=(-torch.log1p(-u)).to("cuda"),
                          tally_len=torch.zeros(M, dtype=torch.float64, device="cuda"),
                          tally_abs=torch.zeros(M, dtype=torch.float64, device="cuda"))


def prepare_buffers(vrt, torch, grid, o, d, rho, spec, mode=None):
    """Output buffers for the workload: windows of the configured size and a
    spill sized up front from spill_chunks_per_ray, doubled until a full step
    fits (set-up; the buffers are then reused)."""
    mode = mode or spec["mode"]
    N = o.shape[0]
    chunks = int(N * spec["spill_chunks_per_ray"]) + 1
    while True:
        bufs = make_buffers(vrt, N, spec, torch, chunks)
        add_transport(bufs, spec, torch, grid.M)
        step(vrt, grid, o, d, rho, bufs, spec, mode)
        torch.cuda.synchronize()
        asked = int(bufs.work[1].item())
        if asked <= chunks:
            return bufs
        chunks = 2 * asked
        del bufs


def step(vrt, grid, o, d, rho, bufs, spec, mode, reuse_order=False):
    """One step of the path: the coherent ray order, then vor_trace (start
    cells, traversal, segment windows and spill). reuse_order: the order and
    the start cells of the previous step on the same rays are reused, so
    only the traversal kernel runs (the roofline launches)."""
    ordered = spec.get("ordered", False)
    if ordered and not reuse_order:
        vrt.order_rays(grid, o, d, bufs.order, bufs.order_ws)
    gd = spec.get("grid_density", True)   # the density bound to the grid at set-up (vor_grid_bind_density)
    opts = vrt.TraceOpts(vrt.MODES[mode], 0, 0.0, 1 if spec.get("persistent", False) else 0,
                         1 if reuse_order else 0, 0, 1 if gd else 0)
    out = bufs.struct(use_order=ordered, **(getattr(bufs, "transport", None) or {}))
    rc = vrt.load().vor_trace(grid.handle, vrt._ptr(o), vrt._ptr(d), o.shape[0], vrt._ptr(None if gd else rho),
                              float(spec.get("kappa", 1.0)), vrt.ctypes.byref(opts), vrt.ctypes.byref(out),
                              vrt._stream())
    if rc != vrt.VOR_OK:
        raise vrt.VorError(rc, "vor_trace")


def run_steps(vrt, torch, grid, o, d, rho, bufs, spec, mode, n, timed, reuse_order=False):
    """Run n steps; with timed=True return per-step milliseconds (HIP events
    on the stream the library launches on, i.e. torch's current stream)."""
    times = []
    stream = torch.cuda.current_stream()
    for _ in range(n):
        if timed:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        step(vrt, grid, o, d, rho, bufs, spec, mode, reuse_order=reuse_order)
        if timed:
            e1.record(stream)
            times.append((e0, e1))
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in times]


def cpu_model() -> str:
    """The host CPU's model name (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, spec, oracle):
    """The oracle (FP64 brute force over all sites) on a bounded sample of
    the same rays (both origin classes in equal parts where the workload has
    two), with all host threads."""
    n = min(spec["cpu_rays"], w.N)
    sub = w.subsample(n, seed=123, split=w.meta.get("n_central"))
    threads = oracle.get_threads()
    t0 = time.perf_counter()
    ref = oracle.trace(w.sites, w.box, w.density, sub.origins, sub.dirs, cap=4096, segments=True)
    dt = time.perf_counter() - t0
    crossings = int(ref["nseg"].sum())
    return sub, ref, dict(value=crossings / dt, unit="crossings/s", cores=threads, kind="oracle",
                          sample=f"{n} of the {w.N} rays (seeded subsample), {crossings} crossings in {dt:.1f} s",
                          host_cpus=os.cpu_count(), cpu_model=cpu_model())


def paper_algorithm_baseline(vrt, torch, grid, w, bufs, oracle, n_max=100_000):
    """The paper's own neighbour-list path loop on the host (oracle/nbtrace.c,
    FP64; Sect. 2.2 with a running point), timed on one core and on all host
    cores, on a seeded sample of the same rays: the like-for-like CPU
    counterpart of the paper's single-core timing (Table 2). Its neighbour
    lists and start cells are those the GPU built and located (the paper
    times the path loop, not the set-up). Also reported: how many rays it
    gives the GPU's segment count (its running point rounds differently, so
    near-ties may resolve otherwise)."""
    n = min(n_max, w.N)
    sub = w.subsample(n, seed=321, split=w.meta.get("n_central"))
    rp, col = grid.neighbors()
    rp, col = rp.cpu().numpy(), col.cpu().numpy()
    start = vrt.locate(grid, sub.origins).cpu().numpy()
    res = {}
    for label, threads in (("one_core", 1), ("all_cores", os.cpu_count() or 1)):
        t0 = time.perf_counter()
        out = oracle.nbtrace(w.sites, w.box, rp, col, w.density, sub.origins, sub.dirs, start, kappa=w.kappa,
                             threads=threads)
        dt = time.perf_counter() - t0
        c = int(out["nseg"].sum())
        res[label] = {"value": c / dt, "unit": "crossings/s", "cores": threads, "ns_per_crossing": dt / c * 1e9,
                      "seconds": dt}
    gpu_n = bufs.n_seg.cpu().numpy()[np.asarray(sub.meta["ray_index"])]
    res.update(kind="the paper's neighbour-list path loop on the host (FP64, running point; neighbour lists and "
                    "start cells from the GPU build), labelled baseline, not the oracle",
               rays=int(n), crossings=int(out["nseg"].sum()), no_exit_events=int(out["fails"].sum()),
               rays_with_the_gpu_count=float(np.mean(out["nseg"] == gpu_n)),
               paper_table2_ns_per_crossing_one_core=[693, 1095])
    return res


def grid_quality(args, torch, vrt, workloads):
    """Grid quality (Sect. 3.3, the Table 1 method): the theoretical density
    rho_t and the gridded density rho_g (the density of the cell that holds
    the point, i.e. at its site) at 10^7 points uniform over the box;
    quality = the standard deviation of rho_t - rho_g. The hot part is
    locating the points (timed with HIP events), with both structures: the
    bucket grid of sites (vor_locate) and the paper's block lists from the
    cells' bounding boxes (vor_locate_blocks, Sect. 2.3); both must give the
    same cell for every point. For each disc the sites drawn from the density
    (the workload's placement) are compared with as many uniform sites. The
    cells of 2000 of the points are checked against the oracle's brute-force
    locate."""
    import oracle
    n_pts = 10_000_000
    out = {}
    for name, cfg in (("exp_disc", 1), ("flared_disc", 2)):
        w = workloads.make_config(cfg)
        field = workloads.DENSITY_FIELDS[name]
        pts = workloads.grid_quality_points(w.box, n_pts)
        rho_t = field(pts)
        dev_pts = torch.as_tensor(pts, device="cuda")
        cell = torch.empty(n_pts, dtype=torch.int32, device="cuda")
        res = {}
        for placement in ("density", "uniform"):
            sites = w.sites if placement == "density" else workloads.uniform_in_box(
                np.random.default_rng(7), w.M, w.box)
            rho_site = field(sites)
            grid = vrt.build_grid(sites, w.box, block_lists=True)
            info = grid.info()

            def timed(fn):
                fn(grid.handle, vrt._ptr(dev_pts), n_pts, vrt._ptr(cell), vrt._stream())
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(3):
                    fn(grid.handle, vrt._ptr(dev_pts), n_pts, vrt._ptr(cell), vrt._stream())
                e1.record()
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / 3

            ms_blocks = timed(vrt.load().vor_locate_blocks)
            c_blocks = cell.cpu().numpy()
            ms = timed(vrt.load().vor_locate)
            c = cell.cpu().numpy()
            diff = rho_t - rho_site[c]
            sample = slice(0, 2_000)
            ref, _ = oracle.locate(sites, w.box, pts[sample])
            nblk = int(np.prod(info["block_dims"]))
            res[placement] = {"sigma": float(diff.std()), "sigma_rel_mean": float(diff.std() / rho_t.mean()),
                              "locate_ms": ms, "points_per_s": n_pts / (ms / 1e3),
                              "oracle_cell_mismatches": int((ref != c[sample]).sum()),
                              "block_lists": {"locate_ms": ms_blocks, "points_per_s": n_pts / (ms_blocks / 1e3),
                                              "blocks": nblk, "mean_cells_per_block": info["block_entries"] / nblk,
                                              "cells_differing_from_vor_locate": int((c_blocks != c).sum())}}
            print(f"[bench] grid quality {name} {placement}: {res[placement]}", file=sys.stderr, flush=True)
            grid.free()
        res["uniform_over_density_sigma"] = res["uniform"]["sigma"] / res["density"]["sigma"]
        out[name] = dict(sites=w.M, points=n_pts, **res)
    best = out["flared_disc"]["density"]["block_lists"]
    result = {"metric": "grid quality: std of rho_t - rho_g at uniform points (Sect. 3.3); locate points/s "
                        "(block lists of Sect. 2.3)",
              "value": best["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": 3, "warmup": 1,
              "ms_per_step": best["locate_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f64", "data": "synthetic",
              "config": {"workload": "grid quality: 10^7 uniform points located on the 10^5-site exponential "
                                     "disc and the 10^6-site flared disc"}, "grids": out}
    print(json.dumps(result), flush=True)


def spill_per_ray(vrt, torch, grid, o, d, stride):
    """Mean spill chunks per ray that paths of these rays need past a window
    of `stride` slots (a tau-only trace of a sample; set-up): sizes the
    first spill pool of each served request."""
    b = vrt.TraceBuffers(o.shape[0], locate_first=True)
    vrt.trace_into(grid, o, d, None, b, mode="mixed", persistent=True)
    torch.cuda.synchronize()
    need = (b.n_seg.long() - stride).clamp(min=0)
    return float(((need + vrt.SPILL_CHUNK - 1) // vrt.SPILL_CHUNK).double().mean())


def request_chunks(n, per_ray):
    """The first spill pool of a request of n rays: 25% over the mean need,
    plus a few chunks (a pool too small costs a second run of the request)."""
    return int(math.ceil(1.25 * per_ray * n)) + 8


def run_server(vrt, grids, rhos, reqs, offsets, stride, budget, keep=False, grid_density=False, per_ray=None):
    """Submit the requests at the given offsets (seconds from the start) to a
    fresh server, reap them in completion order, and return the wall time
    from the first submission to the last completion (each request's
    submission time plus its latency as the server measured it, so that the
    client's reaping -- result copies included -- does not count), crossings,
    p50/p99 latency and (keep) every request's tau and statuses.
    grid_density: the requests use the densities bound to their grids
    instead of rhos. per_ray[g]: mean spill chunks per ray on grid g (the
    requests' first spill pools); every path is stored whole."""
    import threading

    srv = vrt.Server(grids, budget_bytes=budget)
    lat = [None] * len(reqs)
    t_sub = [None] * len(reqs)
    taus = [None] * len(reqs)
    stats = [None] * len(reqs)
    done = threading.Event()
    index = {}

    def reaper():
        nfin = 0
        while nfin < len(reqs):
            rid = srv.next_done(1.0)
            if rid is None:
                continue
            i = index.get(rid)
            while i is None:   # the submitter records the id just after submit returns
                time.sleep(0)
                i = index.get(rid)
            lat[i] = srv.latency(rid)
            if keep:   # the per-ray results (the release below waits for these copies)
                res = srv.result(rid, paths=False)
                taus[i] = res["tau"]
                stats[i] = res["status"]
            srv.release(rid)
            nfin += 1
        done.set()

    th = threading.Thread(target=reaper, daemon=True)
    t0 = time.perf_counter()
    th.start()
    for i, r in enumerate(reqs):
        wait = t0 + offsets[i] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        n = r["o"].shape[0]
        chunks = request_chunks(n, per_ray[r["grid"]]) if stride > 0 else 0
        # no lock around submit: a lock held there kept the reaper from releasing
        # completed requests (and so from returning their memory) while the
        # submissions went on
        t_sub[i] = time.perf_counter()
        rid = srv.submit(r["grid"], r["o"], r["d"], None if grid_density else rhos[r["grid"]], mode=r["mode"],
                         seg_stride=stride, spill_chunks=chunks, grid_density=grid_density)
        index[rid] = i
    if not done.wait(600):
        raise RuntimeError("serving run did not finish within 600 s")
    t1 = max(a + b for a, b in zip(t_sub, lat))   # the last completion
    st = srv.stats()
    while st["running"]:   # crossings are counted when a launch ends
        time.sleep(0.001)
        st = srv.stats()
    srv.close()
    lat = np.array(lat, dtype=np.float64)
    out = dict(seconds=t1 - t0, crossings=st["crossings"], rate=st["crossings"] / (t1 - t0),
               p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
               launches=st["launches"], redecisions=st["fp64_redecisions"], reruns=st["reruns"])
    if keep:
        import torch
        counts = torch.bincount(torch.cat(stats).long(), minlength=5).cpu().tolist()
        if counts[vrt.RAY_OVERFLOW] or counts[vrt.RAY_STEPLIMIT]:
            raise RuntimeError(f"served paths incomplete: status counts {counts}")
        out["status_counts"] = counts
    return (out, taus) if keep else out


def serving(args, torch, vrt, workloads):
    """Serving mix: three resident grids (10^4, 10^5, 10^6 sites shaped like
    the uniform cube, the exponential disc and the flared disc), Poisson
    arrivals of requests with log-uniform sizes in [256, 65536] rays, grid
    chosen uniformly, accuracy class 50/50 FP64/mixed, 1 GiB of output
    budget. First the saturated rate (every request submitted at once), then
    offered loads of 0.5, 0.8 and 0.95 of it; value = crossings/s at 0.8."""
    grids_w = workloads.serving_grids()
    grids = [vrt.build_grid(w.sites, w.box) for w in grids_w]
    rhos = [torch.as_tensor(w.density, device="cuda") for w in grids_w]
    bound = args.serving_density == "grid"
    if bound:
        for g, r in zip(grids, rhos):
            g.bind_density(r)   # set-up: the resident grids hold their density fields
    print(f"[bench] serving grids built: {[g.info()['build_ms'] for g in grids]} ms", file=sys.stderr, flush=True)
    n_req = args.requests
    stride = 32
    budget = int(args.mix_budget_gib * (1 << 30))
    base = workloads.serving_requests(n_req, grids_w, rate_hz=1.0)
    reqs = [dict(grid=r["grid"], mode=["fp64", "mixed"][r["mode"]], o=torch.as_tensor(r["origins"], device="cuda"),
                 d=torch.as_tensor(r["dirs"], device="cuda"), t=r["t"]) for r in base]
    total_rays = sum(r["o"].shape[0] for r in reqs)
    per_ray = []
    for gi, g in enumerate(grids):
        mine = [r for r in reqs if r["grid"] == gi][:40]
        o = torch.cat([r["o"] for r in mine]).contiguous()
        d = torch.cat([r["d"] for r in mine]).contiguous()
        per_ray.append(spill_per_ray(vrt, torch, g, o, d, stride))
    print(f"[bench] spill chunks per ray past {stride}-slot windows: {per_ray}", file=sys.stderr, flush=True)

    def run(offsets, keep=False):
        return run_server(vrt, grids, rhos, reqs, offsets, stride, budget, grid_density=bound, per_ray=per_ray,
                          keep=keep)

    run(np.zeros(len(reqs)))   # warm-up
    sat, _ = run(np.zeros(len(reqs)), keep=True)
    req_rate_sat = len(reqs) / sat["seconds"]
    loads = {}
    for f in (0.5, 0.8, 0.95):
        gaps = np.array([r["t"] for r in reqs]) / (f * req_rate_sat)
        loads[f] = run(gaps)
        print(f"[bench] load {f}: {loads[f]}", file=sys.stderr, flush=True)
    main = loads[0.8]
    result = {
        "metric": METRIC, "value": main["rate"], "unit": "crossings/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": 1, "ms_per_step": main["seconds"] * 1e3 / len(reqs), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 / f32+f64 (50/50 classes)", "data": "synthetic",
        "config": {"workload": f"serving: 3 resident grids (1e4, 1e5, 1e6 sites), {len(reqs)} Poisson requests "
                               f"of 256-65536 rays ({total_rays} rays), 50/50 FP64/mixed, "
                               f"{args.mix_budget_gib:g} GiB output budget, "
                               f"whole paths ({stride}-slot windows and spill chains), "
                               f"offered load 0.8 of saturation, densities "
                               + ("bound to the grids" if bound else "passed per request"), "requests": len(reqs),
                   "rays": total_rays, "seg_stride": stride, "spill_chunks_per_ray_estimate": per_ray},
        "p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"],
        "saturated": sat, "loads": {str(k): v for k, v in loads.items()},
    }
    print(json.dumps(result), flush=True)


def serving_precision_result(torch, vrt, workloads, n_requests, budget_gib, with_load=True):
    """The mixed-precision serving tracer against the plain FP64 GPU tracer on
    the 10^6-site flared disc (the serving mix's large grid). The same
    requests (log-uniform sizes in [256, 65536] rays from random sites,
    isotropic) are served all-FP64 and all-mixed, every request submitted at
    once (saturated) and (with_load) at an offered load of 0.8 of that, with
    whole paths: 32-slot windows and spill chains from each request's pool,
    the density field bound to the resident grid (every leg reads it there).
    Beside them vor_trace runs the same rays in one persistent launch, with
    the same windows and a spill sized for every path, in FP64 and mixed, in
    submission order and in the coherent order of vor_order_rays. Every
    request's tau must be identical between the two serving runs and equal
    to vor_trace's (mixed mode reproduces FP64: equal accuracy), and no
    served ray may end without its whole path. The serving kernel's HBM
    rate is the algorithmic bytes of the same paths (the counters of the
    mixed vor_trace launch, which stores every segment as the server does)
    over the serving wall time."""
    g = workloads.serving_grids()[2]
    grid = vrt.build_grid(g.sites, g.box)
    rho = torch.as_tensor(g.density, device="cuda")
    grid.bind_density(rho)   # a resident grid carries its density field; every leg below reads it there
    stride, budget = 32, int(budget_gib * (1 << 30))
    base = workloads.serving_requests(n_requests, [g], rate_hz=1.0)
    reqs = [dict(grid=0, mode=None, o=torch.as_tensor(r["origins"], device="cuda"),
                 d=torch.as_tensor(r["dirs"], device="cuda"), t=r["t"]) for r in base]
    sizes = [r["o"].shape[0] for r in reqs]
    O = torch.cat([r["o"] for r in reqs]).contiguous()
    D = torch.cat([r["d"] for r in reqs]).contiguous()
    N = O.shape[0]
    per_ray = [spill_per_ray(vrt, torch, grid, O[:200_000], D[:200_000], stride)]
    zeros = np.zeros(len(reqs))
    served, taus = {}, {}
    for mode in ("fp64", "mixed"):
        for r in reqs:
            r["mode"] = mode
        kw = dict(per_ray=per_ray, grid_density=True)
        run_server(vrt, [grid], [rho], reqs, zeros, stride, budget, **kw)   # warm-up
        sat, taus[mode] = run_server(vrt, [grid], [rho], reqs, zeros, stride, budget, keep=True, **kw)
        served[mode] = {"saturated": sat}
        if with_load:
            gaps = np.array([r["t"] for r in reqs]) / (0.8 * len(reqs) / sat["seconds"])
            served[mode]["load_0.8"] = run_server(vrt, [grid], [rho], reqs, gaps, stride, budget, **kw)
        print(f"[bench] serving {mode}: {served[mode]}", file=sys.stderr, flush=True)
    same = all(torch.equal(a, b) for a, b in zip(taus["fp64"], taus["mixed"]))

    # the plain tracer on the same rays, one launch each, whole paths
    plain = {}
    tau_plain = None
    for key, mode, ordered in (("fp64", "fp64", False), ("fp64_ordered", "fp64", True),
                               ("mixed", "mixed", False), ("mixed_ordered", "mixed", True)):
        # densities bound to the grid, as the served requests read them
        spec = {"mode": mode, "stride": stride, "spill_chunks_per_ray": 1.25 * per_ray[0], "persistent": True,
                "grid_density": True, "ordered": ordered}
        bufs = prepare_buffers(vrt, torch, grid, O, D, rho, spec, mode)
        bufs.counters.zero_()
        ms = float(np.mean(run_steps(vrt, torch, grid, O, D, rho, bufs, spec, mode, 3, timed=True)))
        c = bufs.counters.cpu().numpy().astype(np.float64) / 3
        st = np.bincount(bufs.status.cpu().numpy(), minlength=5)
        if st[vrt.RAY_OVERFLOW] or st[vrt.RAY_STEPLIMIT]:
            raise RuntimeError(f"plain tracer output incomplete: {st.tolist()}")
        plain[key] = {"ms": ms, "rate": c[0] / (ms / 1e3), "counters": c}
        if key == "mixed":
            tau_plain = bufs.tau.clone()
        del bufs
    splits = np.cumsum([0] + sizes)
    equal_plain = all(torch.equal(taus["mixed"][i], tau_plain[splits[i]:splits[i + 1]]) for i in range(len(reqs)))
    alg = algorithmic_bytes(plain["mixed"]["counters"], N, "mixed", False)
    sat_m = served["mixed"]["saturated"]
    serving_gbs = alg / sat_m["seconds"] / 1e9
    best_fp64 = max(plain["fp64"]["rate"], plain["fp64_ordered"]["rate"])
    return {
        "rate": sat_m["rate"], "seconds": sat_m["seconds"], "p50_ms": sat_m["p50_ms"], "p99_ms": sat_m["p99_ms"],
        "requests": len(reqs), "rays": N, "budget_gib": budget_gib, "seg_stride": stride,
        "spill_chunks_per_ray_estimate": per_ray[0],
        "served": served,
        "plain_tracer": {m: {"ms": v["ms"], "rate": v["rate"]} for m, v in plain.items()},
        "mixed_serving_over_fp64_serving": sat_m["rate"] / served["fp64"]["saturated"]["rate"],
        "mixed_serving_over_plain_fp64": sat_m["rate"] / plain["fp64"]["rate"],
        "mixed_serving_over_best_plain_fp64": sat_m["rate"] / best_fp64,
        "accuracy": {"tau_identical_fp64_vs_mixed_serving": same, "tau_serving_equals_plain": equal_plain,
                     "overflow_rays": sat_m["status_counts"][vrt.RAY_OVERFLOW] +
                     served["fp64"]["saturated"]["status_counts"][vrt.RAY_OVERFLOW]},
        "roofline": {"bound": "hbm", "achieved": serving_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": serving_gbs / HBM_PEAK_GBS, "algorithmic_bytes": alg},
    }


def serving_precision(args, torch, vrt, workloads):
    """The serving_precision workload on its own line; value = the mixed
    serving rate (saturated)."""
    r = serving_precision_result(torch, vrt, workloads, args.requests, args.budget_gib)
    result = {
        "metric": METRIC, "value": r["rate"], "unit": "crossings/s", "n_gpus": 1, "steps": r["requests"],
        "warmup": 1, "ms_per_step": r["seconds"] * 1e3 / r["requests"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"serving precision: {r['requests']} requests of 256-65536 rays ({r['rays']} rays) "
                               f"on the 1e6-site flared disc, all submitted at once, mixed vs FP64, whole paths, "
                               f"{args.budget_gib:g} GiB output budget",
                   "requests": r["requests"], "rays": r["rays"], "budget_gib": args.budget_gib},
        "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
        "serving_roofline": r["roofline"],
        **{k: v for k, v in r.items() if k not in ("rate", "seconds", "p50_ms", "p99_ms", "roofline")},
    }
    print(json.dumps(result), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)   # p50/p99 over at least 20 calls
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="flared_disc", choices=sorted(WORKLOADS) + ["serving", "serving_precision", "grid_quality"])
    ap.add_argument("--requests", type=int, default=2000, help="serving: number of requests")
    ap.add_argument("--budget-gib", type=float, default=8.0, help="serving_precision: output budget (GiB)")
    ap.add_argument("--mix-budget-gib", type=float, default=1.0, help="serving: output budget (GiB)")
    ap.add_argument("--serving-density", choices=["grid", "array"], default="grid",
                    help="serving: densities bound to the resident grids, or passed with every request")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the exact-output comparison (its extra trace launches would mix into a profile of "
                         "the trace kernel)")
    ap.add_argument("--records", choices=["auto", "fp32", "compact"], default="auto",
                    help="record layout of the traced grids (auto: compact for tables beyond the last-level cache)")
    ap.add_argument("--no-configs", action="store_true",
                    help="default workload only: leave out the other configurations' block")
    ap.add_argument("--config-requests", type=int, default=2000,
                    help="requests of the serving-precision entry of the configurations block")
    ap.add_argument("--roofline-reps", type=int, default=5)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, three elementwise copies of 512 MiB (float64 negation) whose "
                         "hardware counters calibrate the trace kernel's")
    args = ap.parse_args(argv)
    global RECORDS
    RECORDS = args.records

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only: the path is measured on one MI355X "
                                   "(rays would shard across GPUs with the grid replicated on each)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1310_1854_amd import vrt, workloads

    if args.workload == "serving":
        torch.cuda.set_device(0)
        return serving(args, torch, vrt, workloads)
    if args.workload == "serving_precision":
        torch.cuda.set_device(0)
        return serving_precision(args, torch, vrt, workloads)
    if args.workload == "grid_quality":
        torch.cuda.set_device(0)
        return grid_quality(args, torch, vrt, workloads)
    torch.cuda.set_device(0)
    result = measure(args, torch, vrt, workloads, args.workload, args.steps, args.warmup, args.roofline_reps,
                     with_cpu=not args.no_cpu)
    if args.workload == "flared_disc" and not args.no_configs:
        # the other configurations on the same line: their own rates, rooflines and accuracy
        cfgs = {}
        for name in ("exp_disc", "clumpy", "uniform_cube"):
            torch.cuda.empty_cache()
            cfgs[name] = measure(args, torch, vrt, workloads, name, 5, 1, 3, with_cpu=not args.no_cpu,
                                 cpu_rays=WORKLOADS[name]["cpu_rays_configs"])
            print(f"[bench] {name}: {cfgs[name]['value']:.3e} crossings/s", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        cfgs["serving_precision"] = serving_precision_result(torch, vrt, workloads, args.config_requests, 32.0,
                                                             with_load=False)
        print(f"[bench] serving precision: {cfgs['serving_precision']['rate']:.3e} crossings/s", file=sys.stderr,
              flush=True)
        result["configs"] = cfgs
    result["paper_context"] = PAPER_TABLE2
    print(json.dumps(result), flush=True)
    if args.copy_calibration:
        copy_calibration(torch)


# The paper's own timing (Table 2, Sect. 3.4), quoted as context: the time
# per Voronoi cell crossing of its CPU implementation on one core of a
# desktop computer (model not stated), whole photon-shooting phase divided
# by the cells crossed; and the octree grid's time on the same models.
PAPER_TABLE2 = {
    "source": "Table 2 (Sect. 3.4): time per cell crossing, one core of a desktop computer, CPU model and "
              "precision not stated; elapsed time of the whole photon-shooting phase / cells crossed",
    "voronoi_ns_per_crossing": {"torus_monochromatic": 693, "torus_panchromatic": 1006,
                                "spiral_monochromatic": 903, "spiral_panchromatic": 1095},
    "octree_ns_per_crossing": {"torus_monochromatic": 219, "torus_panchromatic": 400,
                               "spiral_monochromatic": 309, "spiral_panchromatic": 442},
    "voronoi_crossings_per_s_one_core": [1e9 / 1095, 1e9 / 693],
    "cells": {"torus": "about 950,000, uniform", "spiral": "about 1,350,000, density-weighted"},
}


def measure(args, torch, vrt, workloads, name, steps, warmup, roofline_reps, with_cpu, cpu_rays=None):
    """One workload of WORKLOADS: warmup, then `steps` timed steps; the trace
    kernel alone for the roofline; FP64 on the same batch; the oracle on a
    sample (with_cpu). Returns the result dict."""
    spec = WORKLOADS[name]
    if cpu_rays is not None:
        spec = dict(spec, cpu_rays=cpu_rays)
    args = argparse.Namespace(**dict(vars(args), workload=name, steps=steps, warmup=warmup,
                                     roofline_reps=roofline_reps, no_cpu=not with_cpu))
    mode = spec["mode"]
    t0 = time.perf_counter()
    w = workloads.make_config(spec["cfg"])
    print(f"[bench] workload {w.name}: {w.M} sites, {w.N} rays ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    grid = build_grid(vrt, w)
    info = grid.info()
    print(f"[bench] grid built in {info['build_ms']:.0f} ms, nnz {info['nnz']}", file=sys.stderr, flush=True)
    o = torch.as_tensor(w.origins, device="cuda").contiguous()
    d = torch.as_tensor(w.dirs, device="cuda").contiguous()
    rho = torch.as_tensor(w.density, device="cuda").contiguous()
    bufs = prepare_buffers(vrt, torch, grid, o, d, rho, spec)

    # warmup, then K timed steps
    run_steps(vrt, torch, grid, o, d, rho, bufs, spec, mode, args.warmup, timed=False)
    bufs.counters.zero_()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    step_ms = run_steps(vrt, torch, grid, o, d, rho, bufs, spec, mode, args.steps, timed=True)
    wall = time.perf_counter() - t_start
    c = bufs.counters.cpu().numpy().astype(np.float64) / max(args.steps, 1)
    status = np.bincount(bufs.status.cpu().numpy(), minlength=5)
    spilled = int(bufs.work[2].item())
    if status[vrt.RAY_OVERFLOW] or status[vrt.RAY_STEPLIMIT]:
        raise SystemExit(f"incomplete output: status counts {status.tolist()}")
    ms_per_step = wall * 1e3 / max(args.steps, 1)
    crossings = c[0]
    value = crossings / (ms_per_step / 1e3)
    print(f"[bench] {mode}: {ms_per_step:.2f} ms/step, {crossings:.0f} crossings/step, {value:.3e}/s, "
          f"spilled rays {spilled}", file=sys.stderr, flush=True)
    tau_mixed = bufs.tau.clone()
    nseg_mixed = bufs.n_seg.clone()

    # the trace kernel alone for the roofline: the same launch with the order
    # and the start cells already computed (events around vor_trace only)
    k_ms = run_steps(vrt, torch, grid, o, d, rho, bufs, spec, mode, 1, timed=False)
    bufs.counters.zero_()
    k_ms = run_steps(vrt, torch, grid, o, d, rho, bufs, spec, mode, args.roofline_reps, timed=True,
                     reuse_order=True)
    kc = bufs.counters.cpu().numpy().astype(np.float64) / args.roofline_reps
    k_avg = float(np.mean(k_ms))
    alg = algorithmic_bytes(kc, w.N, mode, bool(spec.get("transport")))
    achieved = alg / (k_avg / 1e3) / 1e9
    recs_per_step = kc[4] / max(kc[3], 1)

    # FP64 on the same batch: rate, and equality of every ray's result
    fb = prepare_buffers(vrt, torch, grid, o, d, rho, spec, mode="fp64")
    run_steps(vrt, torch, grid, o, d, rho, fb, spec, "fp64", 1, timed=False)
    fb.counters.zero_()
    t1 = time.perf_counter()
    f_ms = run_steps(vrt, torch, grid, o, d, rho, fb, spec, "fp64", max(2, args.steps // 2), timed=True)
    f_wall = (time.perf_counter() - t1) / max(2, args.steps // 2)
    fc = fb.counters.cpu().numpy().astype(np.float64) / max(2, args.steps // 2)
    fp64_value = fc[0] / f_wall
    same_tau = bool(torch.equal(fb.tau, tau_mixed))
    same_nseg = bool(torch.equal(fb.n_seg, nseg_mixed))
    # the bound density against the same field passed as an array (one more step)
    density_check = None
    if spec.get("grid_density", True):
        run_steps(vrt, torch, grid, o, d, rho, bufs, dict(spec, grid_density=False), mode, 1, timed=False)
        density_check = {"tau_bit_identical": bool(torch.equal(bufs.tau, tau_mixed)),
                         "n_seg_identical": bool(torch.equal(bufs.n_seg, nseg_mixed))}

    del fb
    exact = None if (spec.get("transport") or args.no_exact) else \
        exact_output(vrt, torch, grid, o, d, rho, bufs, spec, mode)
    traffic, traffic_src, l2_hit = measured_traffic(args.workload)
    copy_bw = copy_bandwidth(torch)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "crossings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mode == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w.M} sites, {w.N} rays, {mode} mode"
                               + (f", kappa {spec['kappa']}, interaction points and both tallies"
                                  if spec.get("transport") else ""),
                   "sites": w.M, "rays": w.N, "mode": mode, "seg_stride": spec["stride"],
                   "ordered": bool(spec.get("ordered", False)),
                   "persistent": bool(spec.get("persistent", False)),
                   "density": "bound to the grid" if spec.get("grid_density", True) else "array per call",
                   "records": info.get("record_layout")},
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "crossings_per_step": crossings,
        "rays_past_window_per_step": spilled,
        "records_per_step": recs_per_step,
        "lane_utilization": kc[3] / (64.0 * kc[5]) if kc[5] > 0 else None,
        "fp64_redecision_rate": c[2] / max(c[3], 1),
        "fallback_rate": c[1] / max(c[0], 1),
        "eps_mix": 2.0 ** -20,
        "fp64_value": fp64_value,
        "fp64_ms_per_step": f_wall * 1e3,
        "mixed_vs_fp64": {"tau_bit_identical": same_tau, "n_seg_identical": same_nseg},
        "bound_vs_array_density": density_check,
        "exact_output": exact,
        "grid": {"build_ms": info["build_ms"], "nnz": info["nnz"], "max_row": info["max_row"],
                 "device_bytes": info["device_bytes"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_trace_persistent" if spec.get("persistent") else "k_trace",
                     "kernel_avg_ms": k_avg, "algorithmic_bytes": alg, "traffic_source": traffic_src,
                     "kernel_source_sha256_16": kernel_source_hash(), "l2_hit_rate": l2_hit,
                     "copy_bw": copy_bw, "frac_of_copy": achieved / copy_bw},
    }
    if not args.no_cpu:
        import oracle
        sub, ref, cpu = cpu_baseline(w, spec, oracle)
        cpu["paper_algorithm"] = paper_algorithm_baseline(vrt, torch, grid, w, bufs, oracle)
        result["cpu_baseline"] = cpu
        # accuracy on the sample: the same rays through the library
        res = vrt.trace(grid, sub.origins, sub.dirs, w.density, mode=mode, segments="exact")
        tau = res["tau"].cpu().numpy()
        mism = 0
        max_dl = max_dt = 0.0
        for i in range(sub.N):
            if ref["n_near"][i] > 0:
                continue
            cells, lens = vrt.ray_path(res, i)
            n = int(ref["nseg"][i])
            if len(cells) != n or not np.array_equal(cells, ref["seg_cell"][i, :n]):
                mism += 1
                continue
            if n:
                max_dl = max(max_dl, float(np.max(np.abs(lens - ref["seg_len"][i, :n]))) / ref["chord"][i])
            max_dt = max(max_dt, abs(tau[i] - ref["tau"][i]) / max(ref["tau"][i], 1e-300))
        result["accuracy"] = {"oracle_sample_rays": int(sub.N), "near_tie_rays": int((ref["n_near"] > 0).sum()),
                              "cell_sequence_mismatches": mism, "max_len_err_rel_chord": max_dl,
                              "max_tau_err_rel": max_dt}
        if spec.get("transport"):
            from oracle import transport as T
            idx = np.asarray(sub.meta["ray_index"])
            ts = bufs.transport["tau_stop"].cpu().numpy()[idx]
            it = T.interactions(ref, w.density, float(spec["kappa"]), ts)
            g_cell = bufs.stop_cell.cpu().numpy()[idx]
            g_s = bufs.stop_s.cpu().numpy()[idx]
            clean = (ref["n_near"] == 0) & (ref["status"] == 0)
            result["accuracy"]["stop_cell_mismatches"] = int((g_cell != it["cell"])[clean].sum())
            result["accuracy"]["max_stop_s_err_rel_chord"] = float(
                np.max(np.abs(g_s - it["s"])[clean] / ref["chord"][clean])) if clean.any() else 0.0
    if spec.get("transport"):
        result["transport"] = transport_check(vrt, torch, grid, o, d, rho, bufs, spec, mode)
    del bufs
    grid.free()
    return result




def exact_output(vrt, torch, grid, o, d, rho, bufs, spec, mode, reps=3):
    """Every path whole, in compact rows (ray i's segments at
    [ray_off[i], ray_off[i + 1])), two ways, wall time per batch including
    the host's read of the total that sizes the rows: one traversal (a bench
    step into the windows and spill chains), the scan and vor_gather_paths;
    against a tau-only counting pass, the scan and a second traversal that
    writes each segment at its offset. Checks that both give the same rows."""
    N = o.shape[0]
    gd = spec.get("grid_density", True)
    dens = None if gd else rho
    kw = dict(kappa=float(spec.get("kappa", 1.0)), mode=mode, persistent=bool(spec.get("persistent", False)),
              ordered=bool(spec.get("ordered", False)), grid_density=gd)
    one, two = [], []
    cell1 = len1 = None
    count = vrt.TraceBuffers(N, ordered=kw["ordered"])
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(vrt, grid, o, d, rho, bufs, spec, mode)
        off = vrt.exclusive_scan(bufs.n_seg)
        total = int(off[-1].item())
        if cell1 is None:
            cell1 = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
            len1 = torch.empty(max(total, 1), dtype=torch.float64, device="cuda")
        vrt.gather_paths(bufs, off, cell1, len1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        vrt.trace_into(grid, o, d, dens, count, **kw)
        off2 = vrt.exclusive_scan(count.n_seg)
        total2 = int(off2[-1].item())
        if r == 0:
            fill = vrt.TraceBuffers(N, total_segments=max(total2, 1), ordered=kw["ordered"])
        fill.ray_off = off2
        if kw["ordered"]:   # the second traversal reuses the first one's order and start cells
            fill.order.copy_(count.order)
        fill.start_cell.copy_(count.start_cell)
        vrt.trace_into(grid, o, d, dens, fill, start_given=True, **kw)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r > 0:   # the first round allocates
            one.append((t1 - t0) * 1e3)
            two.append((t2 - t1) * 1e3)
    same = total == total2 and bool(torch.equal(off, off2)) and bool(torch.equal(cell1[:total], fill.seg_cell[:total])) \
        and bool(torch.equal(len1[:total], fill.seg_len[:total]))
    del count, fill, cell1, len1
    torch.cuda.empty_cache()
    return {"one_traversal_ms": float(np.median(one)), "two_pass_ms": float(np.median(two)),
            "segments": total, "rows_identical": same,
            "how": "one traversal into windows + spill, scan, vor_gather_paths; vs counting pass, scan, second "
                   "traversal into the offsets reusing the first one's order and start cells (host read of the "
                   "total included in both)"}


def transport_check(vrt, torch, grid, o, d, rho, bufs, spec, mode):
    """One more launch with zeroed tallies: the fraction of packages that
    interact, the absorbed luminosity of all paths against its closed form
    (the sum of 1 - exp(-tau) over the cut paths) and the path-length tally
    against the summed path lengths."""
    tr = bufs.transport
    tr["tally_len"].zero_()
    tr["tally_abs"].zero_()
    step(vrt, grid, o, d, rho, bufs, spec, mode)
    torch.cuda.synchronize()
    ok = bufs.status == 0
    want = float((-torch.expm1(-bufs.tau))[ok].sum())
    got = float(tr["tally_abs"].sum())
    path = float(bufs.stop_s[ok].sum())     # length of every (cut) path: the path-length tally's total
    tl = float(tr["tally_len"].sum())
    return {"kappa": spec["kappa"], "interacting_fraction": float((bufs.stop_cell[ok] >= 0).double().mean()),
            "absorbed_total": got, "absorbed_closed_form": want, "absorbed_rel_err": abs(got - want) / want,
            "tally_len_total": tl, "path_length_total": path, "tally_len_rel_err": abs(tl - path) / path}


def copy_bandwidth(torch, mib: int = 1024, reps: int = 5) -> float:
    """Device copy bandwidth in GB/s (bytes read + written per second) of a
    plain streaming kernel: scaling of mib MiB of float64, event-timed (a
    multiplication, so that the negations of copy_calibration stay apart in
    the counter runs)."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 3.0, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(src, 3.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * n * 8 / (ms / 1e3) / 1e9


def copy_calibration(torch, mib: int = 512, reps: int = 3):
    """A plain streaming kernel of known size: read mib MiB, write mib MiB."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: {reps} x negation of {mib} MiB float64", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
