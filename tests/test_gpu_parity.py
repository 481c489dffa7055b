"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Sizes the oracle finishes in seconds, spanning several blocks and a ragged
tail; the full-size configurations are in test_gpu_fullsize.py. FP64 parity
is expected bit-exact (the FP64 path evaluates the same expressions in the
same order, without FMA contraction); the bar written in the tests is the
stated tolerance (1e-12 relative in FP64 mode, 1e-5 in mixed mode).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.dda import lattice_path
from paper_1310_1854_amd import workloads as W
from pathcmp import compare, gpu_paths

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.fixture(scope="module")
def vrt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1310_1854_amd import vrt as v
    v.load()
    return v


def _geo(grid, w, origins, dirs):
    """What pathcmp needs to check near-tie paths for validity."""
    rp, col = grid.neighbors()
    return dict(sites=w.sites, box=w.box, density=w.density, kappa=w.kappa, origins=origins, dirs=dirs,
                nbr=(rp.cpu().numpy(), col.cpu().numpy()))


def _trace(vrt, grid, w, mode, segments="exact", **kw):
    out = vrt.trace(grid, w.origins, w.dirs, w.density, kappa=w.kappa, mode=mode, segments=segments, **kw)
    return gpu_paths(out)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_golden_hand_paths(vrt, mode):
    g = json.load(open(os.path.join(HERE, "golden", "hand_paths.json")))
    for c in g["cases"]:
        grid = vrt.build_grid(np.array(c["sites"], float), c["box"])
        out = vrt.trace(grid, [c["origin"]], [c["dir"]], np.array(c["density"], float), mode=mode)
        p = gpu_paths(out)
        n = int(p["n_seg"][0])
        assert list(p["seg_cell"][:n]) == c["cells"], c["name"]
        tol = c["rel_tol"] * max(c["chord"], 1.0)
        assert np.allclose(p["seg_len"][:n], c["lengths"], rtol=0, atol=tol), c["name"]
        assert abs(p["tau"][0] - c["tau"]) <= tol * max(1.0, c["tau"]), c["name"]
        assert p["status"][0] == 0


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_cubic_lattice_voxel_walk(vrt, mode):
    w = W.cubic_lattice(8, N=3000)
    grid = vrt.build_grid(w.sites, w.box)
    p = _trace(vrt, grid, w, mode)
    xs, ys, zs = w.meta["xs"], w.meta["ys"], w.meta["zs"]
    for r in range(w.N):
        c, l, L = lattice_path(xs, ys, zs, w.box, w.origins[r], w.dirs[r])
        n = int(p["n_seg"][r])
        o = int(p["ray_off"][r])
        assert list(p["seg_cell"][o:o + n]) == c
        assert np.array_equal(p["seg_len"][o:o + n], np.array(l))   # exact on the dyadic lattice


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_random_tensor_lattice_voxel_walk(vrt, mode):
    w = W.random_tensor_lattice((9, 6, 11), N=3000)
    grid = vrt.build_grid(w.sites, w.box)
    p = _trace(vrt, grid, w, mode)
    for r in range(w.N):
        c, l, L = lattice_path(w.meta["xs"], w.meta["ys"], w.meta["zs"], w.box, w.origins[r], w.dirs[r])
        n = int(p["n_seg"][r])
        o = int(p["ray_off"][r])
        assert list(p["seg_cell"][o:o + n]) == c
        assert np.max(np.abs(p["seg_len"][o:o + n] - np.array(l))) <= TOL[mode] * L


# --------------------------------------------------------------------------
# the small uniform configuration, every ray
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cube(vrt):
    w = W.uniform_cube(M=1000, N=10_000)
    ref = oracle.trace(w.sites, w.box, w.density, w.origins, w.dirs, cap=64)
    return w, vrt.build_grid(w.sites, w.box), ref


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
@pytest.mark.parametrize("segments", ["exact", "stride"])
@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("ordered", [False, True])
def test_uniform_cube_all_rays(vrt, cube, mode, segments, persistent, ordered):
    w, grid, ref = cube
    out = vrt.trace(grid, w.origins, w.dirs, w.density, mode=mode, segments=segments, seg_stride=8,
                    spill_chunks=20000, persistent=persistent, ordered=ordered)
    p = gpu_paths(out)
    if segments == "stride":
        # paths longer than the window continue in their spill chain
        host = {}
        cells, lens, off = [], [], [0]
        for r in range(w.N):
            c, l = vrt.ray_path(out, r, host)
            cells.append(c)
            lens.append(l)
            off.append(off[-1] + len(c))
        p.update(seg_cell=np.concatenate(cells), seg_len=np.concatenate(lens), ray_off=np.array(off))
        assert int(out["work"][2].item()) == int((p["n_seg"] > 8).sum()) > 0
    st = compare(p, ref, TOL[mode], geo=_geo(grid, w, w.origins, w.dirs))
    assert st["clean"] > 0.99 * w.N
    if mode == "fp64":
        assert st["max_len_diff"] == 0.0 and st["max_tau_diff"] == 0.0
    c = out["counters"].cpu().numpy()
    assert c[0] == p["n_seg"].sum()


def test_ray_order_is_a_permutation_and_changes_nothing(vrt):
    import torch
    w = W.flared_disc(M=50_000, N=300_001, seed=21)
    grid = vrt.build_grid(w.sites, w.box)
    o = torch.as_tensor(w.origins, device="cuda")
    d = torch.as_tensor(w.dirs, device="cuda")
    order = torch.empty(w.N, dtype=torch.int32, device="cuda")
    ws = torch.empty(int(vrt.load().vor_order_workspace_bytes(w.N)), dtype=torch.uint8, device="cuda")
    vrt.order_rays(grid, o, d, order, ws)
    ordr = order.cpu().numpy()
    assert np.array_equal(np.sort(ordr), np.arange(w.N))
    a = vrt.trace(grid, o, d, w.density, mode="mixed", segments="stride", seg_stride=32, spill_chunks=200_000)
    b = vrt.trace(grid, o, d, w.density, mode="mixed", segments="stride", seg_stride=32, spill_chunks=200_000,
                  ordered=True)
    for k in ("tau", "n_seg", "status"):
        assert torch.equal(a[k], b[k]), k
    n = w.N
    mask = torch.arange(32, device="cuda")[None, :] < a["n_seg"].clamp(max=32)[:, None]
    assert torch.equal(a["seg_cell"].view(n, 32)[mask], b["seg_cell"].view(n, 32)[mask])
    assert torch.equal(a["seg_len"].view(n, 32)[mask], b["seg_len"].view(n, 32)[mask])
    ha, hb = {}, {}
    for r in np.nonzero(a["n_seg"].cpu().numpy() > 32)[0][:200]:
        ca, la = vrt.ray_path(a, int(r), ha)
        cb, lb = vrt.ray_path(b, int(r), hb)
        assert np.array_equal(ca, cb) and np.array_equal(la, lb)


@pytest.mark.parametrize("n", [16383, 16384])
def test_ray_order_at_the_small_batch_threshold(vrt, n):
    """Below 2^14 rays the order is the identity; from there on it is the
    coherent sort. Either way a permutation that changes no result."""
    import torch
    w = W.exp_disc(M=20_000, N=n, seed=22)
    grid = vrt.build_grid(w.sites, w.box)
    o = torch.as_tensor(w.origins, device="cuda")
    d = torch.as_tensor(w.dirs, device="cuda")
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(int(vrt.load().vor_order_workspace_bytes(n)), dtype=torch.uint8, device="cuda")
    vrt.order_rays(grid, o, d, order, ws)
    ordr = order.cpu().numpy()
    assert np.array_equal(np.sort(ordr), np.arange(n))
    assert np.array_equal(ordr, np.arange(n)) == (n < 1 << 14)
    kw = dict(mode="mixed", segments="exact", persistent=True)
    a = vrt.trace(grid, o, d, w.density, **kw)
    b = vrt.trace(grid, o, d, w.density, ordered=True, **kw)
    for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("persistent", [False, True])
def test_start_cell_pass_changes_nothing(vrt, cube, persistent):
    """Start cells located at each ray's start and in a pass of their own
    (vor_trace_out.start_cell) give identical results, matching the oracle."""
    import torch
    w, grid, ref = cube
    kw = dict(mode="mixed", segments="exact", persistent=persistent, ordered=True)
    a = vrt.trace(grid, w.origins, w.dirs, w.density, locate_first=False, **kw)
    b = vrt.trace(grid, w.origins, w.dirs, w.density, locate_first=True, **kw)
    for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
        assert torch.equal(a[k], b[k]), k
    st = compare(gpu_paths(b), ref, TOL["mixed"])
    assert st["clean"] > 0.99 * w.N


def test_start_cells_reused_across_calls(vrt):
    """A point source (one origin for every ray, in coherent order: one
    cooperative search per wave) plus scattered origins; the start cells of
    the first call, reused by a second call with another kappa
    (opts.start_given), give the same paths and tau scaled by kappa."""
    import torch
    w = W.flared_disc(M=50_000, N=100_000, seed=31)
    grid = vrt.build_grid(w.sites, w.box)
    o = torch.as_tensor(w.origins, device="cuda")
    d = torch.as_tensor(w.dirs, device="cuda")
    rho = torch.as_tensor(w.density, device="cuda")
    ref = vrt.trace(grid, o, d, rho, mode="mixed", segments="none", persistent=True, locate_first=False)
    b = vrt.TraceBuffers(w.N, ordered=True)
    vrt.trace_into(grid, o, d, rho, b, mode="mixed", persistent=True, ordered=True)
    torch.cuda.synchronize()
    assert torch.equal(b.tau, ref["tau"]) and torch.equal(b.n_seg, ref["n_seg"])
    assert torch.equal(b.status, ref["status"])
    tau1 = b.tau.clone()
    vrt.trace_into(grid, o, d, rho, b, kappa=2.0, mode="mixed", persistent=True, ordered=True, start_given=True)
    torch.cuda.synchronize()
    assert torch.equal(b.n_seg, ref["n_seg"])
    assert torch.equal(b.tau, 2.0 * tau1)      # kappa is a power of two: exact
    n_src = int((torch.linalg.norm(o, dim=1) == 0).sum())
    assert n_src > 10_000                       # the point-source half exercises the cooperative search


def test_long_rows_rank_per_lane(vrt):
    """Rows too long for one wave's cooperative ranking (a central cell with
    ~200 faces, every ray starting in it) are ranked per lane; the results
    still equal FP64's and the oracle's."""
    import torch
    rng = np.random.default_rng(41)
    u = rng.normal(size=(200, 3))
    shell = 0.5 * u / np.linalg.norm(u, axis=1)[:, None]
    bg = W.uniform_in_box(rng, 3000, [-1, -1, -1, 1, 1, 1])
    bg = bg[np.linalg.norm(bg, axis=1) > 0.65]
    sites = np.concatenate([[[0.0, 0.0, 0.0]], shell, bg])
    box = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]
    grid = vrt.build_grid(sites, box)
    assert grid.info()["max_row"] >= 150
    n = 4096
    o = np.tile([[1e-3, -2e-3, 5e-4]], (n, 1))
    d = W.isotropic_dirs(rng, n)
    rho = rng.uniform(0.5, 2.0, len(sites))
    a = vrt.trace(grid, o, d, rho, mode="mixed", segments="exact", persistent=True, ordered=True)
    b = vrt.trace(grid, o, d, rho, mode="fp64", segments="exact")
    for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
        assert torch.equal(a[k], b[k]), k
    ref = oracle.trace(sites, box, rho, o[:512], d[:512], cap=64)
    p = gpu_paths(a)
    st = compare(p, ref, TOL["mixed"])      # the first 512 rays
    assert st["clean"] > 0.99 * 512
    assert int(p["seg_cell"][int(p["ray_off"][0])]) == 0     # every path starts in the central cell


def test_no_exit_fallback_recovers(vrt):
    """Sect. 2.2's no-exit fallback: faces removed from the table of some
    cells (vor_grid_truncate_row) make paths through them miss exits; the
    step that then finds the current point beyond a plane advances a small
    distance and locates the point again. Paths that never meet a damaged
    cell are unchanged; the others still end at the wall with status OK and
    their full length (the advances excepted); FP64 and mixed mode take the
    same decisions. (A path left in a wrong cell while moving away from every
    plane it has passed is not caught: the fallback fires on an exit behind
    the current point, so the cells listed after the damage may differ.)"""
    import torch
    w = W.uniform_cube(M=1000, N=10_000, seed=61)
    grid = vrt.build_grid(w.sites, w.box)
    damaged = np.argsort(np.linalg.norm(w.sites, axis=1))[:40]   # cells near the centre
    for s in damaged:
        grid.truncate_row(int(s), 4)
    a = vrt.trace(grid, w.origins, w.dirs, w.density, mode="fp64", segments="exact")
    b = vrt.trace(grid, w.origins, w.dirs, w.density, mode="mixed", segments="exact", persistent=True,
                  ordered=True)
    for k in ("tau", "n_seg", "status", "n_fallback", "ray_off", "seg_cell", "seg_len"):
        assert torch.equal(a[k], b[k]), k
    p = gpu_paths(a)
    ref = oracle.trace(w.sites, w.box, w.density, w.origins, w.dirs, cap=64)
    nfb = p["n_fallback"]
    assert nfb.sum() > 100 and int(a["counters"][1].item()) == nfb.sum()
    assert np.all(p["status"] == 0)
    eps = 1e-12 * float(np.linalg.norm(np.array(w.box[3:]) - np.array(w.box[:3])))
    dset = set(damaged.tolist())
    n_clean = 0
    for r in range(w.N):
        cells, lens = p["seg_cell"][p["ray_off"][r]:p["ray_off"][r + 1]], p["seg_len"][p["ray_off"][r]:p["ray_off"][r + 1]]
        L = ref["chord"][r]
        n = int(ref["nseg"][r])
        if ref["n_near"][r] == 0 and not (set(ref["seg_cell"][r, :n].tolist()) & dset):
            assert nfb[r] == 0 and list(cells) == list(ref["seg_cell"][r, :n])   # never meets a damaged cell
            n_clean += 1
            continue
        # every advance of the fallback is left out of the segments (R6)
        assert abs(lens.sum() + nfb[r] * eps - L) <= 1e-9 * L, r
    assert n_clean > 0.3 * w.N
    # a larger advance (opts.eps_fb): the paths still reach the wall, each advance missing from the lengths
    big = 1e-6
    c = vrt.trace(grid, w.origins, w.dirs, w.density, mode="mixed", segments="exact", persistent=True,
                  ordered=True, eps_fb=big)
    pc = gpu_paths(c)
    assert np.all(pc["status"] == 0) and pc["n_fallback"].sum() > 100
    total = int(pc["ray_off"][-1])
    tot = np.bincount(np.repeat(np.arange(w.N), pc["n_seg"]), weights=pc["seg_len"][:total], minlength=w.N)
    hit = pc["n_fallback"] > 0
    assert np.all(np.abs(tot[hit] + pc["n_fallback"][hit] * big - ref["chord"][hit]) <= 1e-9 * ref["chord"][hit])
    # clean paths do not depend on it
    clean = pc["n_fallback"] == 0
    assert np.array_equal(pc["n_seg"][clean], p["n_seg"][clean])
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(vrt.VorError):
            vrt.trace(grid, w.origins[:10], w.dirs[:10], w.density, segments="none", eps_fb=bad)


def test_grid_from_torch_allocator(vrt):
    """vor_build_grid with a caller allocator (here torch's caching
    allocator through vor_allocator): the grid's memory is torch's, counted
    by it and given back at vor_grid_free, and the grid traces the same
    paths as one built with hipMalloc."""
    import torch
    w = W.exp_disc(M=20_000, N=3000, seed=63)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    alloc = vrt.torch_allocator()
    g1 = vrt.build_grid(w.sites, w.box, block_lists=True, allocator=alloc)
    held = torch.cuda.memory_allocated() - before
    info = g1.info()
    assert held >= 0.9 * info["device_bytes"], (held, info["device_bytes"])
    g0 = vrt.build_grid(w.sites, w.box, block_lists=True)
    for mode in ("fp64", "mixed"):
        a = vrt.trace(g0, w.origins, w.dirs, w.density, mode=mode, segments="exact", persistent=True, ordered=True)
        b = vrt.trace(g1, w.origins, w.dirs, w.density, mode=mode, segments="exact", persistent=True, ordered=True)
        for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
            assert torch.equal(a[k], b[k]), (mode, k)
        del a, b
    r0, c0 = g0.neighbors()
    r1, c1 = g1.neighbors()
    assert torch.equal(r0, r1) and torch.equal(c0, c1)
    torch.cuda.synchronize()
    mid = torch.cuda.memory_allocated()
    g1.free()
    assert mid - torch.cuda.memory_allocated() >= 0.9 * info["device_bytes"]
    g0.free()


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
@pytest.mark.parametrize("persistent", [False, True])
def test_rays_from_outside_enter_the_box(vrt, mode, persistent):
    """opts.enter: rays from outside start where they enter the box
    (distances from the origin); rays that miss it, or point away, are
    OUTSIDE; origins inside are unaffected. Against the oracle's entry."""
    w = W.uniform_cube(M=1000, N=6000, seed=71)
    k = w.dirs / np.linalg.norm(w.dirs, axis=1)[:, None]
    o = w.origins - 4.0 * k                  # outside, heading for the cube
    d = k.copy()
    o[:1000] = w.origins[:1000]              # inside
    d[1000:1500] = -k[1000:1500]             # outside, heading away: misses
    o[1500:1600, 0] = 3.0                    # outside, moving parallel to the x walls: misses
    d[1500:1600, 0] = 0.0
    # origins that are no point (NaN or infinite coordinates): no path, whichever way they head
    bad = [float("nan"), float("inf"), -float("inf")]
    for i in range(1600, 1660):
        o[i, (i // 3) % 3] = bad[i % 3]
    o[1660:1670] = float("nan")
    ref = oracle.trace(w.sites, w.box, w.density, o, d, cap=64, enter=True)
    assert np.all(ref["status"][1600:1670] == oracle.ST_OUTSIDE)
    assert (ref["status"] == oracle.ST_OUTSIDE).sum() >= 670 and (ref["start_s"] > 0).sum() > 4000
    out = vrt.trace(vrt_grid(vrt, w), o, d, w.density, mode=mode, segments="exact", persistent=persistent,
                    ordered=persistent, enter=True)
    p = gpu_paths(out)
    st = compare(p, ref, TOL[mode], geo=_geo(vrt_grid(vrt, w), w, o, d))
    assert st["clean"] > 0.95 * (ref["status"] == 0).sum()
    if mode == "fp64":
        assert st["max_len_diff"] == 0.0 and st["max_tau_diff"] == 0.0
    # interaction where the path starts for tau_stop <= 0: at the entry point
    ts = np.zeros(w.N)
    out = vrt.trace(vrt_grid(vrt, w), o, d, w.density, mode=mode, segments="none", persistent=persistent,
                    enter=True, tau_stop=ts)
    ok = ref["status"] == 0
    assert np.array_equal(out["stop_s"].cpu().numpy()[ok], ref["start_s"][ok])
    assert np.all(out["status"].cpu().numpy()[1600:1670] == oracle.ST_OUTSIDE)
    assert np.all(out["stop_cell"].cpu().numpy()[1600:1670] == -1)


_GRIDS = {}


def vrt_grid(vrt, w):
    key = (w.name, w.M, float(w.sites[0, 0]))
    if key not in _GRIDS:
        _GRIDS[key] = vrt.build_grid(w.sites, w.box)
    return _GRIDS[key]


def test_mixed_equals_fp64_bitwise(vrt):
    w = W.exp_disc(M=20_000, N=200_000, seed=77)
    grid = vrt.build_grid(w.sites, w.box)
    a = vrt.trace(grid, w.origins, w.dirs, w.density, mode="fp64", segments="exact")
    b = vrt.trace(grid, w.origins, w.dirs, w.density, mode="mixed", segments="exact")
    import torch
    for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
        assert torch.equal(a[k], b[k]), k
    assert b["counters"][2].item() > 0      # some steps were re-decided in FP64


def _grazing_dirs(rng, nhat, tilts):
    """Unit directions perpendicular to nhat, tilted towards it by a tilt
    drawn from tilts with a random sign (nhat: unit normals, one a row)."""
    a = rng.normal(size=nhat.shape)
    perp = a - (a * nhat).sum(1, keepdims=True) * nhat
    perp /= np.linalg.norm(perp, axis=1, keepdims=True)
    tilt = tilts[rng.integers(0, len(tilts), len(nhat))] * rng.choice([-1.0, 1.0], len(nhat))
    return np.ascontiguousarray(perp + tilt[:, None] * nhat)


# tilts around the band where the FP32 n.k of a face is not trusted (about
# 1e-6 of |n|) and the one where the FP32 crossing of a face the ray runs
# along is far off and has a wide bound
GRAZING_TILTS = np.array([0.0, 1e-9, 1e-7, 5e-7, 2e-6, 1e-5, 1e-4, 1e-3])


def _mixed_vs_fp64(vrt, grid, w):
    import torch
    a = vrt.trace(grid, w.origins, w.dirs, w.density, mode="fp64", segments="exact")
    b = vrt.trace(grid, w.origins, w.dirs, w.density, mode="mixed", segments="exact")
    for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
        assert torch.equal(a[k], b[k]), k
    return gpu_paths(a), int(b["counters"][2].item())


def test_mixed_equals_fp64_on_grazing_rays(vrt):
    """Rays that run nearly parallel to a face: every step is either decided
    in FP64 or certified by the FP32 bound, so the mixed paths equal the FP64
    ones bit for bit, and the FP64 paths equal the oracle's (Sect. 2.2)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(1310)
    # random sites; each ray starts between a site and its nearest neighbour
    # (a Voronoi neighbour), 1e-9 to 0.1 of their distance off the bisector
    # plane, and runs nearly parallel to that plane
    w = W.uniform_cube(M=3000, N=1, seed=4301)
    _, nb = cKDTree(w.sites).query(w.sites, k=2)
    n_r = 4000
    i = rng.integers(0, w.M, n_r)
    nvec = w.sites[nb[i, 1]] - w.sites[i]
    nhat = nvec / np.linalg.norm(nvec, axis=1, keepdims=True)
    off = 10.0 ** rng.uniform(-9, -1, n_r)
    w.origins = np.ascontiguousarray(w.sites[i] + (0.5 - off)[:, None] * nvec)
    w.dirs = _grazing_dirs(rng, nhat, GRAZING_TILTS)
    grid = vrt.build_grid(w.sites, w.box)
    p, redo = _mixed_vs_fp64(vrt, grid, w)
    assert redo > 0                          # the untrusted band was hit
    ref = oracle.trace(w.sites, w.box, w.density, w.origins, w.dirs, cap=64)
    st = compare(p, ref, TOL["fp64"], geo=_geo(grid, w, w.origins, w.dirs))
    assert st["max_len_diff"] == 0.0 and st["max_tau_diff"] == 0.0
    assert st["clean"] > 0.8 * n_r          # the rest start within 1e-9 of a face (near-ties) ...
    assert st["near_segments"] > 0          # ... and are checked for being correct paths

    # the cubic lattice: rays nearly along its faces from random points
    w = W.cubic_lattice(8, N=3000, seed=4302)
    axes = np.eye(3)[rng.integers(0, 3, w.N)]
    w.dirs = _grazing_dirs(rng, axes, GRAZING_TILTS)
    grid = vrt.build_grid(w.sites, w.box)
    p, redo = _mixed_vs_fp64(vrt, grid, w)
    assert redo > 0
    for r in range(w.N):
        c, l, L = lattice_path(w.meta["xs"], w.meta["ys"], w.meta["zs"], w.box, w.origins[r], w.dirs[r])
        o, n = int(p["ray_off"][r]), int(p["n_seg"][r])
        assert list(p["seg_cell"][o:o + n]) == c, r
        assert np.max(np.abs(p["seg_len"][o:o + n] - np.array(l))) <= 1e-12 * L, r


# --------------------------------------------------------------------------
# locate
# --------------------------------------------------------------------------

@pytest.mark.parametrize("cfg", ["cube", "disc"])
def test_locate_matches_oracle(vrt, cfg):
    w = W.uniform_cube(M=3000, N=1, seed=5) if cfg == "cube" else W.exp_disc(M=30_000, N=1, seed=6)
    pts = W.uniform_in_box(np.random.default_rng(9), 20_011, w.box)
    pts = np.concatenate([pts, w.sites[:500], [[w.box[3] + 1, 0, 0], [0, 0, w.box[2] - 1e-9]]])
    grid = vrt.build_grid(w.sites, w.box)
    cell = vrt.locate(grid, pts).cpu().numpy()
    ref, gap = oracle.locate(w.sites, w.box, pts)
    assert np.array_equal(cell, ref)        # equal distances also go to the lowest index on both sides
    assert list(cell[-2:]) == [-1, -1]
    assert np.array_equal(cell[20_011:20_511], np.arange(500))


# --------------------------------------------------------------------------
# the paper's locate structure: cell bounding boxes and block lists
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["cube", "disc", "lattice"])
def test_bboxes_vs_oracle(vrt, case):
    w = {"cube": lambda: W.uniform_cube(M=2000, N=1, seed=61),
         "disc": lambda: W.exp_disc(M=3000, N=1, seed=62),
         "lattice": lambda: W.random_tensor_lattice((6, 5, 7), N=1)}[case]()
    grid = vrt.build_grid(w.sites, w.box, block_lists=True)
    got = grid.bboxes().cpu().numpy()
    _, _, want = oracle.faces(w.sites, w.box, np.arange(w.M), bboxes=True)
    ext = want[:, 3:] - want[:, :3]
    tol = 1e-10 * ext.max(1, keepdims=True) + 1e-13 * (w.box[3:] - w.box[:3]).max()
    assert np.all(np.abs(got[:, :3] - want[:, :3]) <= tol)
    assert np.all(np.abs(got[:, 3:] - want[:, 3:]) <= tol)
    info = grid.info()
    assert info["block_entries"] >= w.M and min(info["block_dims"]) >= 1


def _locate_points(w, rng, n=20000):
    """Uniform points, the sites themselves, points on the bisector plane of
    a site and its nearest neighbour (ties), the box's corners and faces
    (the box is closed) and points outside."""
    from scipy.spatial import cKDTree
    lo, hi = w.box[:3], w.box[3:]
    mids = np.zeros((0, 3))
    if w.M >= 2:
        _, nb = cKDTree(w.sites).query(w.sites, k=2)
        mids = 0.5 * (w.sites + w.sites[nb[:, 1]])
    corners = np.array([[(hi if (c >> a) & 1 else lo)[a] for a in range(3)] for c in range(8)])
    face = rng.uniform(lo, hi, (200, 3))
    ax = rng.integers(0, 3, 200)
    face[np.arange(200), ax] = np.where(rng.random(200) < 0.5, lo[ax], hi[ax])
    outside = rng.uniform(lo - (hi - lo), hi + (hi - lo), (500, 3))
    return np.concatenate([rng.uniform(lo, hi, (n, 3)), w.sites, mids, corners, face, outside])


@pytest.mark.parametrize("occ", [0.25, 1.0, 8.0])
@pytest.mark.parametrize("case", ["cube", "disc", "lattice", "one"])
def test_locate_blocks_matches_oracle(vrt, case, occ):
    rng = np.random.default_rng(63)
    w = {"cube": lambda: W.uniform_cube(M=1500, N=1, seed=64),
         "disc": lambda: W.exp_disc(M=20000, N=1, seed=65),
         "lattice": lambda: W.cubic_lattice(6, N=1),
         "one": lambda: W.uniform_cube(M=1, N=1, seed=66)}[case]()
    grid = vrt.build_grid(w.sites, w.box, block_lists=True, block_occupancy=occ)
    pts = _locate_points(w, rng)
    if case == "lattice":   # points on the cell walls and edges: exact ties between lattice cells
        pts = np.concatenate([pts, rng.integers(0, 7, (3000, 3)).astype(float),
                              rng.integers(0, 13, (3000, 3)) * 0.5])
    got = vrt.locate_blocks(grid, pts).cpu().numpy()
    want, _ = oracle.locate(w.sites, w.box, pts)
    assert np.array_equal(got, want)
    assert np.array_equal(got, vrt.locate(grid, pts).cpu().numpy())


@pytest.mark.parametrize("persistent", [False, True])
def test_trace_with_block_lists_changes_nothing(vrt, persistent):
    """A grid with block lists locates the start cells through them; every
    output equals the trace on the same grid without them."""
    import torch
    w = W.flared_disc(M=20000, N=20000, seed=68)
    o = w.origins.copy()
    o[:500] = w.origins[:500] + 3000.0 * w.dirs[:500]   # from outside, entering
    kw = dict(mode="mixed", segments="exact", persistent=persistent, ordered=True, enter=True)
    a = vrt.trace(vrt.build_grid(w.sites, w.box), o, w.dirs, w.density, **kw)
    b = vrt.trace(vrt.build_grid(w.sites, w.box, block_lists=True), o, w.dirs, w.density, **kw)
    for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
        assert torch.equal(a[k], b[k]), k
    assert int((a["status"] == 0).sum()) > 19000


def test_locate_blocks_needs_the_lists(vrt):
    w = W.uniform_cube(M=100, N=1, seed=67)
    grid = vrt.build_grid(w.sites, w.box)
    assert grid.info()["block_entries"] == 0
    for call in (lambda: vrt.locate_blocks(grid, w.sites), grid.bboxes):
        with pytest.raises(vrt.VorError) as e:
            call()
        assert e.value.code == vrt.VOR_EINVAL


def test_grid_quality_measure(vrt):
    """The grid-quality measure of Sect. 3.3 (std of rho_t - rho_g at uniform
    points, rho_g the density of the cell holding the point) from the GPU's
    locate equals the oracle's exactly; sites drawn from the density
    represent it better than as many uniform sites."""
    sig = {}
    for placement in ("density", "uniform"):
        w = W.exp_disc(M=20_000, N=1, seed=91)
        sites = w.sites if placement == "density" else W.uniform_in_box(np.random.default_rng(5), w.M, w.box)
        pts = W.grid_quality_points(w.box, 20_000, seed=92)
        rho_t = W.exp_disc_density(pts)
        rho_s = W.exp_disc_density(sites)
        cell = vrt.locate(vrt.build_grid(sites, w.box), pts).cpu().numpy()
        ref, _ = oracle.locate(sites, w.box, pts)
        assert np.array_equal(cell, ref)
        sig[placement] = float(np.std(rho_t - rho_s[cell]))
    assert sig["density"] < sig["uniform"]


# --------------------------------------------------------------------------
# neighbour lists against the oracle's brute-force faces
# --------------------------------------------------------------------------

def _rows(rp, col, i):
    return set(col[rp[i]:rp[i + 1]].tolist())


@pytest.mark.parametrize("case", ["cube", "disc_small", "lattice"])
def test_cell_volumes_vs_oracle(vrt, case):
    """Cell volumes from the builder's polyhedra against the oracle's
    (clipped face polygons), and their sum against the box."""
    if case == "cube":
        w = W.uniform_cube(M=1500, N=1, seed=12)
    elif case == "disc_small":
        w = W.flared_disc(M=3000, N=1, seed=13)
    else:
        w = W.cubic_lattice(5, N=1)
    grid = vrt.build_grid(w.sites, w.box)
    vol = grid.volumes().cpu().numpy()
    _, ref = oracle.faces(w.sites, w.box, np.arange(w.M), cap=512)
    box = np.asarray(w.box, float)
    total = float(np.prod(box[3:] - box[:3]))
    assert abs(vol.sum() - total) <= 1e-10 * total
    assert np.max(np.abs(vol - ref) / ref) <= 1e-9
    if case == "lattice":
        assert np.allclose(vol, total / w.M, rtol=1e-12, atol=0)   # every lattice cell is the same cuboid


@pytest.mark.parametrize("case", ["cube", "disc_small", "lattice"])
def test_neighbour_lists_vs_oracle_faces(vrt, case):
    if case == "cube":
        w = W.uniform_cube(M=1500, N=1, seed=12)
    elif case == "disc_small":
        w = W.flared_disc(M=3000, N=1, seed=13)
    else:
        w = W.cubic_lattice(5, N=1)
    grid = vrt.build_grid(w.sites, w.box)
    rp, col = grid.neighbors()
    rp, col = rp.cpu().numpy(), col.cpu().numpy()
    res, vol = oracle.faces(w.sites, w.box, np.arange(w.M), cap=512)
    ext = w.box[3:] - w.box[:3]
    for i in range(w.M):
        got = _rows(rp, col, i)
        nb, ar = res[i]
        scale2 = (vol[i] ** (1.0 / 3.0)) ** 2
        real = set(int(j) for j, a in zip(nb, ar) if a > 1e-9 * scale2)
        anyc = set(int(j) for j in nb)
        assert real <= got, f"cell {i}: missing {real - got}"
        # every listed entry is a contact the brute force also sees, or a
        # degenerate (zero-area) contact at a shared edge or vertex
        extra = got - anyc
        for j in extra:
            assert j >= 0
            d = np.linalg.norm(w.sites[j] - w.sites[i])
            assert d < 4 * np.linalg.norm(ext)
    # symmetric
    for i in range(w.M):
        for j in _rows(rp, col, i):
            if j >= 0:
                assert i in _rows(rp, col, j)
    info = grid.info()
    assert info["nnz_with_walls"] == len(col)


def test_lattice_neighbours_are_the_six_faces(vrt):
    n = 6
    w = W.cubic_lattice(n, N=1)
    grid = vrt.build_grid(w.sites, w.box)
    rp, col = grid.neighbors()
    rp, col = rp.cpu().numpy(), col.cpu().numpy()
    for idx in range(w.M):
        i, j, k = idx // (n * n), (idx // n) % n, idx % n
        want = set()
        for a, (c, lo_wall) in enumerate(((i, -1), (j, -3), (k, -5))):
            step = (n * n, n, 1)[a]
            want.add(idx - step if c > 0 else lo_wall)
            want.add(idx + step if c < n - 1 else lo_wall - 1)
        assert _rows(rp, col, idx) == want


def test_mean_neighbours_uniform(vrt):
    w = W.uniform_cube(M=200_000, N=1, seed=14)
    grid = vrt.build_grid(w.sites, w.box)
    rp, col = grid.neighbors()
    rp, col = rp.cpu().numpy(), col.cpu().numpy()
    far = np.nonzero(np.all(np.abs(w.sites) < 0.8, axis=1))[0]
    counts = np.array([np.sum(col[rp[i]:rp[i + 1]] >= 0) for i in far[:20000]])
    assert abs(counts.mean() - 15.54) < 0.1, counts.mean()


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------

def test_edge_cases(vrt):
    import torch
    box = [-1, -1, -1, 1, 1, 1]
    # one site: one segment of length L
    g1 = vrt.build_grid([[0.1, 0.2, 0.3]], box)
    out = gpu_paths(vrt.trace(g1, [[0, 0, 0], [0.5, 0.5, 0.5]], [[1, 0, 0], [0, 0, -2]], [3.0]))
    assert list(out["n_seg"]) == [1, 1]
    assert np.allclose(out["seg_len"], [1.0, 1.5], rtol=0, atol=1e-15)
    assert np.allclose(out["tau"], [3.0, 4.5], rtol=1e-15)
    # statuses: outside, zero direction, NaN direction, on the wall heading out
    sites = W.uniform_cube(M=50, N=1, seed=3).sites
    g = vrt.build_grid(sites, box)
    o = [[2, 0, 0], [0, 0, 0], [0, 0, 0], [1, 0, 0], [1, 0, 0]]
    d = [[1, 0, 0], [0, 0, 0], [np.nan, 1, 0], [1, 0, 0], [-1, 0, 0]]
    for mode in ("fp64", "mixed"):
        p = gpu_paths(vrt.trace(g, o, d, np.ones(50), mode=mode))
        assert list(p["status"]) == [vrt.RAY_OUTSIDE, vrt.RAY_BADDIR, vrt.RAY_BADDIR, 0, 0]
        assert list(p["n_seg"][:4]) == [0, 0, 0, 0] and p["n_seg"][4] > 0
        assert p["tau"][3] == 0.0
        ref = oracle.trace(sites, box, np.ones(50), o, d, cap=64)
        assert list(ref["status"]) == list(p["status"])
    # no rays
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    p = vrt.trace(g, e, e, None, segments="none")
    assert p["tau"].numel() == 0
    # stride window too small and no spill: overflow status, full count and tau
    w = W.uniform_cube(M=2000, N=500, seed=4)
    g2 = vrt.build_grid(w.sites, w.box)
    full = gpu_paths(vrt.trace(g2, w.origins, w.dirs, w.density))
    small = gpu_paths(vrt.trace(g2, w.origins, w.dirs, w.density, segments="stride", seg_stride=3))
    # and with a spill too small for the longest paths
    tiny = gpu_paths(vrt.trace(g2, w.origins, w.dirs, w.density, segments="stride", seg_stride=3, spill_chunks=1))
    assert np.array_equal(tiny["n_seg"], full["n_seg"]) and np.array_equal(tiny["tau"], full["tau"])
    assert (tiny["status"] == vrt.RAY_OVERFLOW).sum() >= 1
    assert np.array_equal(small["n_seg"], full["n_seg"]) and np.array_equal(small["tau"], full["tau"])
    over = full["n_seg"] > 3
    assert over.any() and np.all(small["status"][over] == vrt.RAY_OVERFLOW)
    assert np.all(small["status"][~over] == 0)
    # tau-only mode agrees with segment mode
    only = gpu_paths(vrt.trace(g2, w.origins, w.dirs, w.density, segments="none"))
    assert np.array_equal(only["tau"], full["tau"]) and np.array_equal(only["n_seg"], full["n_seg"])


def _degenerate_case(name, rng):
    """(sites, box) of a geometrically degenerate grid."""
    if name == "coplanar":        # every site in z = 0: the cells are prisms
        xy = rng.uniform(-1, 1, (300, 2))
        return np.column_stack([xy, np.zeros(300)]), np.array([-1.0, -1, -1, 1, 1, 1])
    if name == "collinear":       # every site on the x axis: the cells are slabs
        return np.column_stack([np.sort(rng.uniform(-1, 1, 40)), np.zeros(40), np.zeros(40)]), \
            np.array([-1.0, -1, -1, 1, 1, 1])
    if name == "walls":           # sites on the walls, edges and corners of the box
        p = rng.uniform(-1, 1, (400, 3))
        ax = rng.integers(0, 3, 400)
        p[np.arange(400), ax] = np.where(rng.random(400) < 0.5, -1.0, 1.0)
        corners = np.array([[x, y, z] for x in (-1.0, 1.0) for y in (-1.0, 1.0) for z in (-1.0, 1.0)])
        return np.concatenate([p, corners]), np.array([-1.0, -1, -1, 1, 1, 1])
    if name == "offset":          # a unit box far from the origin
        c = 1e6
        return c + rng.uniform(-1, 1, (500, 3)), np.array([c - 1, c - 1, c - 1, c + 1, c + 1, c + 1])
    if name == "tiny":            # a box of side 1e-6
        return rng.uniform(0, 1e-6, (500, 3)), np.array([0.0, 0, 0, 1e-6, 1e-6, 1e-6])
    if name == "flat":            # a box 10^6 times longer than it is thick
        box = np.array([0.0, 0, 0, 1000, 1, 1e-3])
        return rng.uniform(box[:3], box[3:], (500, 3)), box
    raise ValueError(name)


@pytest.mark.parametrize("name", ["coplanar", "collinear", "walls", "offset", "tiny", "flat"])
def test_degenerate_geometry(vrt, name):
    import torch
    rng = np.random.default_rng(90 + len(name))
    sites, box = _degenerate_case(name, rng)
    M, N = len(sites), 3000
    dens = rng.uniform(0.5, 2.0, M)
    o = rng.uniform(box[:3], box[3:], (N, 3))
    o[:200] = sites[rng.integers(0, M, 200)]                    # from sites
    d = rng.normal(size=(N, 3))
    d[200:400] = np.eye(3)[rng.integers(0, 3, 200)] * rng.choice([-1.0, 1.0], (200, 1))   # along the axes
    grid = vrt.build_grid(sites, box, block_lists=True)
    ref = oracle.trace(sites, box, dens, o, d, cap=1024)
    assert not np.any(ref["status"] == oracle.ST_OVERFLOW)
    a = vrt.trace(grid, o, d, dens, mode="fp64", segments="exact")
    st = compare(gpu_paths(a), ref, TOL["fp64"])
    assert st["max_len_diff"] == 0.0 and st["max_tau_diff"] == 0.0
    assert st["clean"] > 0.5 * N
    for persistent in (False, True):
        b = vrt.trace(grid, o, d, dens, mode="mixed", segments="exact", persistent=persistent, ordered=persistent)
        for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
            assert torch.equal(a[k], b[k]), (k, persistent)
    pts = np.concatenate([rng.uniform(box[:3], box[3:], (5000, 3)), sites])
    want, _ = oracle.locate(sites, box, pts)
    assert np.array_equal(vrt.locate_blocks(grid, pts).cpu().numpy(), want)
    assert np.array_equal(vrt.locate(grid, pts).cpu().numpy(), want)
    vol = grid.volumes().cpu().numpy()
    assert abs(vol.sum() - np.prod(box[3:] - box[:3])) <= 1e-9 * np.prod(box[3:] - box[:3])


def test_build_errors(vrt):
    box = [-1, -1, -1, 1, 1, 1]
    with pytest.raises(vrt.VorError) as e:
        vrt.build_grid([[0, 0, 0], [0.5, 0, 0], [0, 0, 0]], box)
    assert e.value.code == vrt.VOR_EDUP
    with pytest.raises(vrt.VorError) as e:
        vrt.build_grid([[0, 0, 0], [1.5, 0, 0]], box)
    assert e.value.code == vrt.VOR_EOUTSIDE
    with pytest.raises(vrt.VorError) as e:
        vrt.build_grid([[0, 0, 0], [np.nan, 0, 0]], box)
    assert e.value.code == vrt.VOR_EOUTSIDE
    with pytest.raises(vrt.VorError) as e:
        vrt.build_grid([[0, 0, 0]], [0, 0, 0, 0, 1, 1])
    assert e.value.code == vrt.VOR_EINVAL


@pytest.mark.parametrize("n", [0, 1, 1023, 1024, 2047, 2048, 2049, 65535, 65536, 65537, 1_000_003])
def test_exclusive_scan(vrt, n):
    import torch
    rng = np.random.default_rng(n)
    c = rng.integers(0, 100, n).astype(np.int32)
    off = vrt.exclusive_scan(torch.as_tensor(c, device="cuda")).cpu().numpy()
    assert off.shape == (n + 1,)
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(c, dtype=np.int64)]))


def test_ragged_sizes_and_site_permutation(vrt):
    """Several ragged batch sizes through one grid; permuting the site order
    permutes the cell indices and changes nothing else."""
    w = W.uniform_cube(M=777, N=3001, seed=31)
    g = vrt.build_grid(w.sites, w.box)
    ref = gpu_paths(vrt.trace(g, w.origins, w.dirs, w.density))
    for n in (1, 63, 64, 65, 255, 257, 3001):
        p = gpu_paths(vrt.trace(g, w.origins[:n], w.dirs[:n], w.density))
        assert np.array_equal(p["n_seg"], ref["n_seg"][:n])
        assert np.array_equal(p["tau"], ref["tau"][:n])
    perm = np.random.default_rng(2).permutation(w.M)
    inv = np.argsort(perm)
    g2 = vrt.build_grid(w.sites[perm], w.box)
    p2 = gpu_paths(vrt.trace(g2, w.origins, w.dirs, w.density[perm]))
    assert np.array_equal(p2["n_seg"], ref["n_seg"])
    assert np.array_equal(p2["seg_len"], ref["seg_len"])
    assert np.array_equal(p2["seg_cell"], inv[ref["seg_cell"]])
    assert np.array_equal(p2["tau"], ref["tau"])


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_every_store_path_gives_the_exact_paths(vrt, cube, mode):
    """Segment windows of every kind hold the same paths as the exact CSR
    output: strides that are multiples of 8 (cells stored 8 at a time where
    the kernel does so, lengths 4 at a time, the rest written when the path
    ends), a multiple of 4 only and an odd one (one segment at a time), each
    with paths longer than the window continuing in their spill chain."""
    w, grid, _ = cube
    n = 3000
    o, d = w.origins[:n], w.dirs[:n]
    ex = vrt.trace(grid, o, d, w.density, mode=mode, segments="exact", persistent=True, ordered=True)
    ns = ex["n_seg"].cpu().numpy()
    off = ex["ray_off"].cpu().numpy()
    cells = ex["seg_cell"].cpu().numpy()
    lens = ex["seg_len"].cpu().numpy()
    assert len(set((ns % 8).tolist())) == 8          # every count of cells left over at the end
    for stride in (8, 12, 16, 24, 7):
        out = vrt.trace(grid, o, d, w.density, mode=mode, segments="stride", seg_stride=stride,
                        spill_chunks=20000, persistent=True, ordered=True)
        import torch
        assert torch.equal(out["tau"], ex["tau"]) and torch.equal(out["n_seg"], ex["n_seg"])
        assert int(out["work"][2].item()) == int((ns > stride).sum()) > 0
        host = {}
        for r in range(n):
            c, l = vrt.ray_path(out, r, host)
            assert np.array_equal(c, cells[off[r]:off[r + 1]]), (stride, r)
            assert np.array_equal(l, lens[off[r]:off[r + 1]]), (stride, r)


def _host_paths(out, n):
    """Every ray's (cells, lengths) of a stride-window trace result: its
    window, then its spill chain (arrays copied to the host once)."""
    stride = out["seg_stride"]
    ns = out["n_seg"].cpu().numpy()
    wc = out["seg_cell"].cpu().numpy()[:n * stride].reshape(n, stride)
    wl = out["seg_len"].cpu().numpy()[:n * stride].reshape(n, stride)
    first = out["spill_first"].cpu().numpy()
    nxt = out["spill_next"].cpu().numpy()
    sc, sl = out["spill_cell"].cpu().numpy(), out["spill_len"].cpu().numpy()
    ch = 64
    paths = []
    for r in range(n):
        k = int(ns[r])
        cs, ls = [wc[r, :min(k, stride)]], [wl[r, :min(k, stride)]]
        c, left = int(first[r]), k - stride
        while left > 0:
            assert c >= 0, r
            m = min(left, ch)
            cs.append(sc[c * ch:c * ch + m])
            ls.append(sl[c * ch:c * ch + m])
            left -= m
            c = int(nxt[c])
        paths.append((np.concatenate(cs), np.concatenate(ls)))
    return paths


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_store_groups_on_long_paths(vrt, mode):
    """Paths of about 30 segments (a 10^5-site cube) through windows of 16,
    32, 40 and 48 slots: cells stored 16 at a time on 16-slot windows (also
    beyond the first group of a window), 8 at a time on 8-slot ones, every
    count of cells left over at a path's end (mod 16), and paths past the
    window continuing in spill chains -- all equal to the exact CSR output."""
    import torch
    w = W.uniform_cube(M=100_000, N=4000, seed=4311)
    grid = vrt_grid(vrt, w)
    ex = vrt.trace(grid, w.origins, w.dirs, w.density, mode=mode, segments="exact", persistent=True, ordered=True)
    ns = ex["n_seg"].cpu().numpy()
    off = ex["ray_off"].cpu().numpy()
    cells = ex["seg_cell"].cpu().numpy()
    lens = ex["seg_len"].cpu().numpy()
    assert len(set((ns % 16).tolist())) == 16          # every count of cells held back at the end
    for stride in (16, 32, 40, 48):
        out = vrt.trace(grid, w.origins, w.dirs, w.density, mode=mode, segments="stride", seg_stride=stride,
                        spill_chunks=20000, persistent=True, ordered=True)
        assert torch.equal(out["tau"], ex["tau"]) and torch.equal(out["n_seg"], ex["n_seg"])
        assert int(out["work"][2].item()) == int((ns > stride).sum()) > 0
        for r, (c, l) in enumerate(_host_paths(out, w.N)):
            assert np.array_equal(c, cells[off[r]:off[r + 1]]), (stride, r)
            assert np.array_equal(l, lens[off[r]:off[r + 1]]), (stride, r)


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_exact_paths_from_one_traversal(vrt, mode):
    """segments="exact" traces once into windows and spill chains and then
    gathers every path into compact rows (vor_gather_paths, one wave per
    ray). It must give the two-pass route's rows bit for bit: with windows
    that most paths outgrow, with a first spill too small (traced again with
    the spill it asked for) and with windows few paths outgrow; and the
    oracle's paths on a sample."""
    import torch
    w = W.flared_disc(M=20_000, N=20_000, seed=83)
    grid = vrt.build_grid(w.sites, w.box)
    kw = dict(kappa=w.kappa, mode=mode, persistent=True, ordered=True)
    a = vrt.trace(grid, w.origins, w.dirs, w.density, segments="exact_two_pass", **kw)
    ns = a["n_seg"].cpu().numpy()
    assert (ns > 16).mean() > 0.5 and (ns > 64).sum() > 0
    for stride, chunks in ((16, 0), (16, 1), (64, 0), (8, 3)):
        b = vrt.trace(grid, w.origins, w.dirs, w.density, segments="exact", seg_stride=stride, spill_chunks=chunks,
                      **kw)
        for k in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
            assert torch.equal(a[k], b[k]), (k, stride, chunks)
        assert b.get("seg_stride", 0) == 0
    ref = oracle.trace(w.sites, w.box, w.density, w.origins[:300], w.dirs[:300], cap=1024)
    st = compare(gpu_paths(b), ref, TOL[mode])
    assert st["clean"] > 0.9 * 300 and st["max_len_diff"] <= TOL[mode]


def test_gather_paths_without_spill(vrt):
    """vor_gather_paths on windows that hold every path (no spill arrays):
    the rows equal the exact layout's."""
    import torch
    w = W.uniform_cube(M=2000, N=5000, seed=84)
    grid = vrt.build_grid(w.sites, w.box)
    ex = vrt.trace(grid, w.origins, w.dirs, w.density, mode="mixed", segments="exact_two_pass")
    stride = int(ex["n_seg"].max().item())
    o = torch.as_tensor(w.origins, device="cuda")
    d = torch.as_tensor(w.dirs, device="cuda")
    rho = torch.as_tensor(w.density, device="cuda")
    b = vrt.TraceBuffers(w.N, seg_stride=stride)
    vrt.trace_into(grid, o, d, rho, b, mode="mixed")
    off = vrt.exclusive_scan(b.n_seg)
    total = int(off[-1].item())
    cell = torch.empty(total, dtype=torch.int32, device="cuda")
    length = torch.empty(total, dtype=torch.float64, device="cuda")
    vrt.gather_paths(b, off, cell, length)
    torch.cuda.synchronize()
    assert torch.equal(off, ex["ray_off"]) and torch.equal(cell, ex["seg_cell"]) and torch.equal(length, ex["seg_len"])
