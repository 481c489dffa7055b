"""Grids with compact neighbour records (8-byte fixed-point offsets, built
with records="compact"): mixed mode over them must give exactly the FP64
paths, bit for bit, as over the 12-byte FP32 records -- the quantisation of
the offsets is covered by the certified bound or sends the step to FP64.
Cases: every launch shape on the uniform cube (and the oracle), the
exponential disc, the clumpy medium (cells of very different sizes side by
side), grazing rays, cells whose neighbours lie 2^-24 to 1 of the largest
offset away (offsets that round to a few units or to nothing), the
degenerate geometries, the no-exit fallback, transport outputs, rays from
outside and the path server."""
import numpy as np
import pytest

import oracle
from paper_1310_1854_amd import workloads as W
from pathcmp import compare, gpu_paths
from test_gpu_parity import GRAZING_TILTS, _degenerate_case, _geo, _grazing_dirs

pytestmark = pytest.mark.gpu

KEYS = ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len")


@pytest.fixture(scope="module")
def vrt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1310_1854_amd import vrt as v
    v.load()
    return v


def _same(a, b, keys=KEYS, what=""):
    import torch
    for k in keys:
        assert torch.equal(a[k], b[k]), (k, what)


def _fp64_vs_compact(vrt, sites, box, o, d, dens, **kw):
    """FP64 over the default grid against mixed mode over a compact grid
    (one-pass and persistent launches); returns the FP64 result and the
    FP64 re-decisions of the compact launches."""
    g = vrt.build_grid(sites, box)
    gc = vrt.build_grid(sites, box, records="compact")
    assert gc.info()["record_layout"] == "compact"
    a = vrt.trace(g, o, d, dens, mode="fp64", segments="exact", **kw)
    redo = 0
    for persistent in (False, True):
        b = vrt.trace(gc, o, d, dens, mode="mixed", segments="exact", persistent=persistent, ordered=persistent,
                      **kw)
        _same(a, b, what=f"persistent={persistent}")
        redo += int(b["counters"][2].item())
    return a, redo


def test_layout_choice_and_size(vrt):
    w = W.uniform_cube(M=2000, N=1, seed=5)
    g = vrt.build_grid(w.sites, w.box)
    gf = vrt.build_grid(w.sites, w.box, records="fp32")
    gc = vrt.build_grid(w.sites, w.box, records="compact")
    assert g.info()["record_layout"] == "fp32"         # small tables stay FP32 by default
    assert gf.info()["record_layout"] == "fp32"
    i, ic = g.info(), gc.info()
    assert ic["nnz"] == i["nnz"] and ic["max_row"] == i["max_row"]
    # 12 bytes per neighbour become 8 + 4 (record + block offset) less the FP32 record's 4: about 4 bytes each
    assert i["device_bytes"] - ic["device_bytes"] > 3 * i["nnz"] - 8 * w.M
    for k in (g, gc):
        rp, col = k.neighbors()
        assert rp.cpu().numpy().tolist() == gf.neighbors()[0].cpu().numpy().tolist()
    with pytest.raises(ValueError):
        vrt.build_grid(w.sites, w.box, records="fp16")


@pytest.mark.parametrize("segments", ["exact", "stride"])
@pytest.mark.parametrize("persistent", [False, True])
def test_uniform_cube_against_fp32_records_and_oracle(vrt, segments, persistent):
    w = W.uniform_cube(M=3000, N=20_000, seed=41)
    g = vrt.build_grid(w.sites, w.box, records="fp32")
    gc = vrt.build_grid(w.sites, w.box, records="compact")
    kw = dict(kappa=w.kappa, mode="mixed", segments=segments, persistent=persistent, ordered=persistent)
    a = vrt.trace(g, w.origins, w.dirs, w.density, **kw)
    b = vrt.trace(gc, w.origins, w.dirs, w.density, **kw)
    if segments == "exact":
        _same(a, b)
    else:   # the windows' slots past each path's end are not written
        import torch
        _same(a, b, ("tau", "n_seg", "status"))
        stride = a["seg_stride"]
        assert int(a["n_seg"].max().item()) <= stride
        used = torch.arange(stride, device="cuda")[None, :] < a["n_seg"][:, None]
        for k in ("seg_cell", "seg_len"):
            x, y = a[k].view(-1, stride), b[k].view(-1, stride)
            assert torch.equal(x[used], y[used]), k
    if segments == "exact":
        ref = oracle.trace(w.sites, w.box, w.density, w.origins[:2000], w.dirs[:2000], cap=256)
        st = compare(gpu_paths(b), ref, 1e-12)
        assert st["max_len_diff"] == 0.0 and st["clean"] > 0.99 * 2000


def test_exp_disc_and_clumpy_equal_fp64(vrt):
    w = W.exp_disc(M=20_000, N=100_000, seed=77)
    _, redo = _fp64_vs_compact(vrt, w.sites, w.box, w.origins, w.dirs, w.density, kappa=w.kappa)
    assert redo > 0
    w = W.clumpy(M=60_000, N=40_000, seed=78)
    _fp64_vs_compact(vrt, w.sites, w.box, w.origins, w.dirs, w.density, kappa=w.kappa)


def test_neighbours_far_below_the_cell_scale(vrt):
    """Cells next to a tight cluster: their neighbour offsets run from the
    largest down to about 2^-22 of it, so the smallest round to a few units
    of the cell's scale or to nothing; the paths still equal FP64's."""
    rng = np.random.default_rng(2024)
    box = np.array([-1.0, -1, -1, 1, 1, 1])
    coarse = rng.uniform(-1, 1, (400, 3))
    clusters = []
    for s in (1e-3, 1e-3, 1e-5, 1e-5, 1e-7, 1e-7):   # clusters of 16 sites, 1e-3 to 1e-7 across
        c = rng.uniform(-0.5, 0.5, 3)
        clusters.append(c + s * rng.uniform(-1, 1, (16, 3)))
    sites = np.concatenate([coarse] + clusters)
    M, N = len(sites), 6000
    dens = rng.uniform(0.5, 2.0, M)
    o = rng.uniform(-1, 1, (N, 3))
    tgt = np.concatenate(clusters)[rng.integers(0, 96, N)]
    d = tgt - o                            # every ray through a cluster
    d[: N // 3] = rng.normal(size=(N // 3, 3))
    o[N // 2:] = tgt[N // 2:] + 1e-9 * rng.normal(size=(N - N // 2, 3))   # and from inside them
    a, redo = _fp64_vs_compact(vrt, sites, box, o, d, dens)
    assert redo > 0
    ref = oracle.trace(sites, box, dens, o[:1500], d[:1500], cap=1024)
    st = compare(gpu_paths(a), ref, 1e-12)
    assert st["max_len_diff"] == 0.0


def test_grazing_rays_equal_fp64(vrt):
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(1311)
    w = W.uniform_cube(M=3000, N=1, seed=4303)
    _, nb = cKDTree(w.sites).query(w.sites, k=2)
    n_r = 4000
    i = rng.integers(0, w.M, n_r)
    nvec = w.sites[nb[i, 1]] - w.sites[i]
    nhat = nvec / np.linalg.norm(nvec, axis=1, keepdims=True)
    off = 10.0 ** rng.uniform(-9, -1, n_r)
    o = np.ascontiguousarray(w.sites[i] + (0.5 - off)[:, None] * nvec)
    d = _grazing_dirs(rng, nhat, GRAZING_TILTS)
    a, redo = _fp64_vs_compact(vrt, w.sites, w.box, o, d, w.density)
    assert redo > 0
    g = vrt.build_grid(w.sites, w.box)
    ref = oracle.trace(w.sites, w.box, w.density, o, d, cap=64)
    st = compare(gpu_paths(a), ref, 1e-12, geo=_geo(g, w, o, d))
    assert st["max_len_diff"] == 0.0 and st["clean"] > 0.8 * n_r
    # the cubic lattice, rays nearly along its faces
    w = W.cubic_lattice(8, N=3000, seed=4304)
    axes = np.eye(3)[rng.integers(0, 3, w.N)]
    d = _grazing_dirs(rng, axes, GRAZING_TILTS)
    _fp64_vs_compact(vrt, w.sites, w.box, w.origins, d, w.density)


@pytest.mark.parametrize("name", ["coplanar", "collinear", "walls", "offset", "tiny", "flat"])
def test_degenerate_geometry_equal_fp64(vrt, name):
    rng = np.random.default_rng(190 + len(name))
    sites, box = _degenerate_case(name, rng)
    M, N = len(sites), 3000
    dens = rng.uniform(0.5, 2.0, M)
    o = rng.uniform(box[:3], box[3:], (N, 3))
    o[:200] = sites[rng.integers(0, M, 200)]
    d = rng.normal(size=(N, 3))
    d[200:400] = np.eye(3)[rng.integers(0, 3, 200)] * rng.choice([-1.0, 1.0], (200, 1))
    _fp64_vs_compact(vrt, sites, box, o, d, dens)


def test_fallback_on_compact_blocks(vrt):
    """Faces dropped from some cells (vor_grid_truncate_row) on both layouts:
    the same fallbacks and paths."""
    w = W.uniform_cube(M=1000, N=10_000, seed=61)
    g = vrt.build_grid(w.sites, w.box, records="fp32")
    gc = vrt.build_grid(w.sites, w.box, records="compact")
    damaged = np.argsort(np.linalg.norm(w.sites, axis=1))[:40]
    for s in damaged:
        g.truncate_row(int(s), 4)
        gc.truncate_row(int(s), 4)
    kw = dict(mode="mixed", segments="exact", persistent=True, ordered=True)
    a = vrt.trace(g, w.origins, w.dirs, w.density, **kw)
    b = vrt.trace(gc, w.origins, w.dirs, w.density, **kw)
    _same(a, b, KEYS + ("n_fallback",))
    c = vrt.trace(gc, w.origins, w.dirs, w.density, mode="fp64", segments="exact")
    _same(a, c, KEYS + ("n_fallback",))
    assert int(a["n_fallback"].sum().item()) > 100


@pytest.mark.parametrize("grid_density", [False, True])
def test_transport_and_entry_equal_fp64(vrt, grid_density):
    import torch
    w = W.exp_disc(M=20_000, N=30_000, seed=79)
    rng = np.random.default_rng(5)
    o = w.origins.copy()
    o[:3000] = rng.uniform(-30, 30, (3000, 3))            # many from outside the box
    tau_stop = torch.as_tensor(rng.exponential(1.0, w.N), device="cuda")
    weight = torch.as_tensor(rng.uniform(0.5, 1.5, w.N), device="cuda")
    g = vrt.build_grid(w.sites, w.box)
    gc = vrt.build_grid(w.sites, w.box, records="compact")
    dens = w.density
    if grid_density:
        rho = torch.as_tensor(w.density, device="cuda")
        g.bind_density(rho)
        gc.bind_density(rho)
        dens = None
    kw = dict(kappa=w.kappa, segments="exact", tau_stop=tau_stop, weight=weight, tallies=True, enter=True,
              grid_density=grid_density)
    a = vrt.trace(g, o, w.dirs, dens, mode="fp64", **kw)
    for persistent in (False, True):
        b = vrt.trace(gc, o, w.dirs, dens, mode="mixed", persistent=persistent, ordered=persistent, **kw)
        _same(a, b, KEYS + ("stop_cell", "stop_s"), f"persistent={persistent}")
        for k in ("tally_len", "tally_abs"):   # atomics: the order of the sums may differ
            assert torch.allclose(a[k], b[k], rtol=1e-12, atol=1e-300), k


def test_server_over_a_compact_grid(vrt):
    """The path server with requests on an FP32 and a compact grid of the
    same sites, in both precisions: every result equals the plain trace."""
    import torch
    w = W.exp_disc(M=20_000, N=40_000, seed=80)
    g = vrt.build_grid(w.sites, w.box)
    gc = vrt.build_grid(w.sites, w.box, records="compact")
    o = torch.as_tensor(w.origins, device="cuda")
    d = torch.as_tensor(w.dirs, device="cuda")
    rho = torch.as_tensor(w.density, device="cuda")
    want = vrt.trace(g, o, d, rho, kappa=w.kappa, mode="fp64", segments="exact")
    srv = vrt.Server([g, gc], budget_bytes=1 << 30)
    try:
        reqs = []
        for gi in (0, 1):
            for mode in ("fp64", "mixed"):
                for a, b in ((0, 15_000), (15_000, 40_000)):
                    rid = srv.submit(gi, o[a:b], d[a:b], rho, kappa=w.kappa, mode=mode, seg_stride=16)
                    reqs.append((rid, a, b))
        for rid, a, b in reqs:
            srv.wait(rid)
            res = srv.result(rid)
            assert torch.equal(res["tau"], want["tau"][a:b])
            assert torch.equal(res["n_seg"], want["n_seg"][a:b])
            assert torch.equal(res["status"], want["status"][a:b])
            lo, hi = int(want["ray_off"][a]), int(want["ray_off"][b])
            assert torch.equal(res["seg_cell"], want["seg_cell"][lo:hi])
            assert torch.equal(res["seg_len"], want["seg_len"][lo:hi])
            srv.release(rid)
    finally:
        srv.close()


def test_tiny_grids_with_compact_records(vrt):
    """One, two and three sites (cells with no or few neighbours) on compact
    records: mixed mode equals FP64 and the oracle."""
    rng = np.random.default_rng(31)
    box = np.array([-1.0, -1, -1, 1, 1, 1])
    for sites in (np.array([[0.1, 0.2, 0.3]]), np.array([[-0.5, 0, 0], [0.5, 0, 0]]),
                  rng.uniform(-1, 1, (3, 3))):
        o = rng.uniform(-1, 1, (500, 3))
        d = rng.normal(size=(500, 3))
        dens = rng.uniform(0.5, 2.0, len(sites))
        a, _ = _fp64_vs_compact(vrt, sites, box, o, d, dens)
        ref = oracle.trace(sites, box, dens, o, d, cap=16)
        st = compare(gpu_paths(a), ref, 1e-12)
        assert st["max_len_diff"] == 0.0
