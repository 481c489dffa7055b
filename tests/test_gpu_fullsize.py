"""Full-size parity: each configuration at its full size, traced in the
launch configuration bench.py times (mode, stride window, spill,
persistent), checked against the oracle on a seeded sample of rays and by
properties that hold for every ray (total length = chord, statuses, mixed
equal to FP64 segment for segment, consecutive cells are listed
neighbours). Samples: 10^4 rays on the exponential disc, 2x10^3 on the
flared disc (10^3 from the central source, 10^3 from sites), 500 on the
clumpy medium; near-tie rays in them are checked for being one of the
correct paths."""
import time

import numpy as np
import pytest

import bench
import oracle
from paper_1310_1854_amd import workloads as W
from pathcmp import compare

pytestmark = pytest.mark.gpu

SAMPLE = {"exp_disc": 10_000, "flared_disc": 2_000, "clumpy": 500}
TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.fixture(scope="module")
def vrt():
    import torch
    assert torch.cuda.is_available()
    from paper_1310_1854_amd import vrt as v
    v.load()
    return v


@pytest.mark.parametrize("name", ["exp_disc", "flared_disc", "clumpy"])
def test_full_size_in_bench_configuration(vrt, name):
    import torch
    spec = bench.WORKLOADS[name]
    w = W.make_config(spec["cfg"])
    print(f"[fullsize] {name}: {w.M} sites, {w.N} rays", flush=True)
    grid = bench.build_grid(vrt, w)
    o = torch.as_tensor(w.origins, device="cuda").contiguous()
    d = torch.as_tensor(w.dirs, device="cuda").contiguous()
    rho = torch.as_tensor(w.density, device="cuda").contiguous()
    bufs = bench.prepare_buffers(vrt, torch, grid, o, d, rho, spec)
    status = bufs.status.cpu().numpy()
    assert np.all(status == 0), np.bincount(status).tolist()
    n_seg = bufs.n_seg
    stride = spec["stride"]

    # every ray: the segments add up to the chord (window, then spill chain).
    # The spill is re-run with zeroed chunks so that unwritten slots add 0.
    bufs.spill_len.zero_()
    bench.step(vrt, grid, o, d, rho, bufs, spec, spec["mode"])
    torch.cuda.synchronize()
    k = d / torch.linalg.norm(d, dim=1, keepdim=True)
    lo = torch.as_tensor(w.box[:3], device="cuda")
    hi = torch.as_tensor(w.box[3:], device="cuda")
    inf = torch.full_like(k, float("inf"))
    t_hi = torch.where(k > 0, (hi - o) / k, inf)
    t_lo = torch.where(k < 0, (lo - o) / k, inf)
    L = torch.minimum(t_hi.min(dim=1).values, t_lo.min(dim=1).values)
    slots = torch.arange(stride, device="cuda")[None, :]
    win = bufs.seg_len.view(w.N, stride)
    tot = torch.empty(w.N, dtype=torch.float64, device="cuda")
    for a in range(0, w.N, 1 << 20):
        b = min(w.N, a + (1 << 20))
        part = win[a:b]
        tot[a:b] = torch.where(slots < n_seg[a:b, None], part, torch.zeros_like(part)).sum(dim=1)
    del win
    past = torch.nonzero(n_seg > stride).flatten()
    assert int(bufs.work[2].item()) == past.numel()
    chunk_sum = bufs.spill_len.view(-1, 64).sum(dim=1)
    cur = bufs.spill_first[past]
    assert bool((cur >= 0).all())
    extra = torch.zeros(past.numel(), dtype=torch.float64, device="cuda")
    nxt = bufs.spill_next.long()
    while bool((cur >= 0).any()):
        ok = cur >= 0
        extra[ok] += chunk_sum[cur[ok]]
        cur = torch.where(ok, nxt[cur.clamp(min=0)], cur)
    tot[past] += extra
    rel = (tot - L).abs() / L.clamp_min(1e-300)
    assert float(rel.max()) <= 1e-12, float(rel.max())

    # mixed mode returns exactly the FP64 results on every ray, segment for segment (exact rows)
    if spec["mode"] == "mixed":
        kw = dict(segments="exact", persistent=True, ordered=True)
        a = vrt.trace(grid, o, d, rho, mode="fp64", **kw)
        b = vrt.trace(grid, o, d, rho, mode="mixed", **kw)
        torch.cuda.synchronize()
        assert torch.equal(a["tau"], bufs.tau) and torch.equal(a["n_seg"], bufs.n_seg)
        for key in ("tau", "n_seg", "status", "ray_off", "seg_cell", "seg_len"):
            assert torch.equal(a[key], b[key]), key
        del a, b

    # a seeded sample against the oracle, segment by segment
    split = w.meta.get("n_central")
    sub = w.subsample(SAMPLE[name], seed=99, split=split)
    ridx = sub.meta["ray_index"]
    t0 = time.perf_counter()
    ref = oracle.trace(w.sites, w.box, w.density, sub.origins, sub.dirs, cap=8192)
    print(f"[fullsize] {name}: oracle on {sub.N} rays, {int(ref['nseg'].sum())} crossings, "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    n_all = n_seg.cpu().numpy()
    res = dict(n_seg=bufs.n_seg, seg_cell=bufs.seg_cell, seg_len=bufs.seg_len, seg_stride=stride,
               ray_off=torch.arange(0, (w.N + 1) * stride, stride, device="cuda"), spill_first=bufs.spill_first,
               spill_next=bufs.spill_next, spill_cell=bufs.spill_cell, spill_len=bufs.spill_len)
    host = {}
    cells, lens, off = [], [], [0]
    for r in ridx:
        c, l = vrt.ray_path(res, int(r), host)
        cells.append(c)
        lens.append(l)
        off.append(off[-1] + len(c))
    p = dict(tau=bufs.tau.cpu().numpy()[ridx], n_seg=n_all[ridx], status=status[ridx],
             seg_cell=np.concatenate(cells), seg_len=np.concatenate(lens), ray_off=np.array(off))
    rp, col = grid.neighbors()
    rp, col = rp.cpu().numpy(), col.cpu().numpy()
    geo = dict(sites=w.sites, box=w.box, density=w.density, kappa=w.kappa, origins=sub.origins, dirs=sub.dirs,
               nbr=(rp, col))
    st = compare(p, ref, TOL[spec["mode"]], geo=geo)
    print(f"[fullsize] {name}: {st}", flush=True)
    assert st["clean"] >= 0.9 * len(ridx)
    if split is not None:   # both origin classes are in the sample
        assert (ridx < split).sum() == len(ridx) // 2

    # consecutive cells of the sampled paths free of near-ties are neighbours in the grid's lists
    for i, c in enumerate(cells):
        if ref["n_near"][i] == 0:
            for a, b in zip(c[:-1], c[1:]):
                assert b in col[rp[a]:rp[a + 1]]


def test_locate_blocks_full_size(vrt):
    """The paper's block-list locate on the 10^6-site flared disc: the same
    cell as the bucket-grid locate for 2x10^6 uniform points and every site,
    and the oracle's cell on a sample."""
    w = W.make_config(2)
    grid = vrt.build_grid(w.sites, w.box, block_lists=True)
    rng = np.random.default_rng(71)
    pts = np.concatenate([rng.uniform(w.box[:3], w.box[3:], (2_000_000, 3)), w.sites])
    a = vrt.locate_blocks(grid, pts).cpu().numpy()
    b = vrt.locate(grid, pts).cpu().numpy()
    assert np.array_equal(a, b)
    assert np.array_equal(a[2_000_000:], np.arange(w.M))
    ref, _ = oracle.locate(w.sites, w.box, pts[:2000])
    assert np.array_equal(a[:2000], ref)
