"""Serving: resident grids, budgeted admission, continuous batching.

Each request's result must be the same alone and in a mix of requests on
different grids and precision classes, and the same as vor_trace of the
same rays; admission never exceeds the budget; a request that can never
fit is rejected; requests are admitted first-in-first-out."""
import time

import numpy as np
import pytest

from paper_1310_1854_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1310_1854_amd import vrt
    vrt.load()
    ws = [W.uniform_cube(M=10_000, N=1, seed=401), W.exp_disc(M=100_000, N=1, seed=402),
          W.flared_disc(M=200_000, N=1, seed=403)]
    grids = [vrt.build_grid(w.sites, w.box) for w in ws]
    rhos = [torch.as_tensor(w.density, device="cuda") for w in ws]
    return vrt, torch, ws, grids, rhos


def _requests(ws, n_req, seed, lo=256, hi=8192):
    import torch
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        g = int(rng.integers(0, len(ws)))
        w = ws[g]
        n = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        if g == 0:
            o = W.uniform_in_box(rng, n, w.box)
        else:
            o = np.ascontiguousarray(w.sites[rng.integers(0, w.M, n)])
        d = W.isotropic_dirs(rng, n)
        reqs.append(dict(grid=g, mode=["fp64", "mixed"][int(rng.integers(0, 2))],
                         o=torch.as_tensor(o, device="cuda"), d=torch.as_tensor(d, device="cuda")))
    return reqs


def _same(a, b):
    """Equal per-ray results and equal segments in every written slot (slots
    past a ray's count are not written and hold whatever was there)."""
    import torch
    if not all(torch.equal(a[k], b[k]) for k in ("tau", "n_seg", "status")):
        return False
    stride = a["seg_stride"]
    n = a["tau"].numel()
    mask = torch.arange(stride, device="cuda")[None, :] < a["n_seg"].clamp(max=stride)[:, None]
    return all(torch.equal(a[k].view(n, stride)[mask], b[k].view(n, stride)[mask]) for k in ("seg_cell", "seg_len"))


def _idle_stats(srv, timeout=60.0):
    """Server statistics once no launch is in flight (crossings are counted
    when a launch ends, which can be after its requests completed)."""
    t0 = time.time()
    while True:
        st = srv.stats()
        if st["running"] == 0 or time.time() - t0 > timeout:
            return st
        time.sleep(0.001)


def test_alone_equals_in_the_mix_equals_vor_trace(env):
    vrt, torch, ws, grids, rhos = env
    reqs = _requests(ws, 24, seed=5)
    stride = 96
    srv = vrt.Server(grids, budget_bytes=2 << 30)
    try:
        alone = []
        for r in reqs:
            rid = srv.submit(r["grid"], r["o"], r["d"], rhos[r["grid"]], mode=r["mode"], seg_stride=stride)
            srv.wait(rid, 120)
            alone.append(srv.result(rid))
            srv.release(rid)
        ids = [srv.submit(r["grid"], r["o"], r["d"], rhos[r["grid"]], mode=r["mode"], seg_stride=stride)
               for r in reqs]
        for rid in ids:
            srv.wait(rid, 120)
        mixed = [srv.result(rid) for rid in ids]
        torch.cuda.synchronize()
        for rid in ids:
            srv.release(rid)
        st = _idle_stats(srv)
    finally:
        srv.close()
    for r, a, m in zip(reqs, alone, mixed):
        assert _same(a, m)
        ref = vrt.trace(grids[r["grid"]], r["o"], r["d"], rhos[r["grid"]], mode=r["mode"], segments="stride",
                        seg_stride=stride)
        assert torch.equal(ref["tau"], a["tau"]) and torch.equal(ref["n_seg"], a["n_seg"])
        assert torch.equal(ref["status"], a["status"])
        # the first min(n_seg, stride) slots of every ray agree
        ns = a["n_seg"].clamp(max=stride)
        mask = torch.arange(stride, device="cuda")[None, :] < ns[:, None]
        n = r["o"].shape[0]
        assert torch.equal(ref["seg_cell"].view(n, stride)[mask], a["seg_cell"].view(n, stride)[mask])
        assert torch.equal(ref["seg_len"].view(n, stride)[mask], a["seg_len"].view(n, stride)[mask])
    assert st["completed"] == 2 * len(reqs)
    assert st["crossings"] == 2 * sum(int(a["n_seg"].sum()) for a in alone)


def test_budget_admission_and_rejection(env):
    vrt, torch, ws, grids, rhos = env
    reqs = _requests(ws, 40, seed=6, lo=2000, hi=20000)
    stride = 64
    per_ray = 8 + 4 + 1 + stride * 12
    budget = 30_000 * per_ray + (1 << 20)   # room for about one large request at a time
    srv = vrt.Server(grids, budget_bytes=budget)
    try:
        big = torch.zeros((200_000, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(vrt.VorError) as e:
            srv.submit(0, big, big, None, seg_stride=stride)
        assert e.value.code == vrt.VOR_EBUDGET
        ids = [srv.submit(r["grid"], r["o"], r["d"], rhos[r["grid"]], mode=r["mode"], seg_stride=stride)
               for r in reqs]
        done = [False] * len(ids)
        order = []
        t0 = time.time()
        while not all(done):
            st = srv.stats()
            assert st["used_bytes"] <= budget
            for i, rid in enumerate(ids):
                if not done[i] and srv.poll(rid):
                    done[i] = True
                    order.append(i)
                    srv.release(rid)
            assert time.time() - t0 < 120, "requests starved"
            time.sleep(0.001)
        assert srv.stats()["used_bytes"] == 0
    finally:
        srv.close()
    # first in, first admitted: completion order never runs far ahead of submission order
    assert max(abs(a - b) for a, b in zip(order, range(len(order)))) < len(order)


def test_server_argument_errors(env):
    vrt, torch, ws, grids, rhos = env
    srv = vrt.Server(grids[:1], budget_bytes=1 << 24)
    try:
        o = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(vrt.VorError):
            srv.submit(3, o, o)                       # no such grid
        rid = srv.submit(0, o, o, None, seg_stride=4)  # zero directions: BADDIR rays
        srv.wait(rid, 30)
        res = srv.result(rid)
        assert np.all(res["status"].cpu().numpy() == vrt.RAY_BADDIR)
        srv.release(rid)
        with pytest.raises(vrt.VorError):
            srv.release(rid)                          # already released
    finally:
        srv.close()


def test_completion_queue_and_early_completion(env):
    """next_done hands out every request once, in completion order; a small
    request launched with large ones completes before they do; a result read
    as soon as its request is done equals vor_trace."""
    vrt, torch, ws, grids, rhos = env
    stride = 32
    rng = np.random.default_rng(11)
    w = ws[2]
    sizes = [200_000, 200_000, 300, 200_000, 500]
    reqs = []
    for n in sizes:
        o = torch.as_tensor(np.ascontiguousarray(w.sites[rng.integers(0, w.M, n)]), device="cuda")
        d = torch.as_tensor(W.isotropic_dirs(rng, n), device="cuda")
        reqs.append((o, d))
    srv = vrt.Server(grids, budget_bytes=2 << 30)
    try:
        ids = [srv.submit(2, o, d, rhos[2], mode="mixed", seg_stride=stride) for o, d in reqs]
        seen = []
        got = {}
        while len(seen) < len(ids):
            rid = srv.next_done(60)
            assert rid is not None, "no request completed within 60 s"
            assert rid not in seen
            seen.append(rid)
            got[rid] = srv.result(rid)      # read while other requests may still run
        assert sorted(seen) == sorted(ids)
        assert srv.next_done(0.01) is None
        lat = {rid: srv.latency(rid) for rid in ids}
        for rid in ids:
            srv.release(rid)
        st = _idle_stats(srv)
    finally:
        srv.close()
    # requests of one launch complete in any order; the small ones need not wait for the large ones
    small = [ids[2], ids[4]]
    large = [ids[0], ids[1], ids[3]]
    assert min(lat[r] for r in small) <= max(lat[r] for r in large)
    for (o, d), rid in zip(reqs, ids):
        ref = vrt.trace(grids[2], o, d, rhos[2], mode="mixed", segments="stride", seg_stride=stride)
        a = got[rid]
        assert torch.equal(ref["tau"], a["tau"]) and torch.equal(ref["n_seg"], a["n_seg"])
        assert torch.equal(ref["status"], a["status"])
        n = o.shape[0]
        mask = torch.arange(stride, device="cuda")[None, :] < a["n_seg"].clamp(max=stride)[:, None]
        assert torch.equal(ref["seg_cell"].view(n, stride)[mask], a["seg_cell"].view(n, stride)[mask])
        assert torch.equal(ref["seg_len"].view(n, stride)[mask], a["seg_len"].view(n, stride)[mask])
    assert st["completed"] == len(ids) and st["running"] == 0


def test_release_waits_for_copies(env):
    """Outputs copied with vor_server_copy_result and released at once stay
    intact until the copy has run. The budget holds one request, the copy
    stream is held back by a bounded spin kernel, and the next request needs
    the same memory: it is admitted only after the copy, so the copy reads
    the first request's results."""
    vrt, torch, ws, grids, rhos = env
    w = ws[2]
    rng = np.random.default_rng(12)
    n, stride = 20000, 16

    def rays():
        o = np.ascontiguousarray(w.sites[rng.integers(0, w.M, n)])
        return torch.as_tensor(o, device="cuda"), torch.as_tensor(W.isotropic_dirs(rng, n), device="cuda")

    (oa, da), (ob, db) = rays(), rays()
    one = n * (8 + 4 + 1) + n * stride * (4 + 8) + 4096
    srv = vrt.Server(grids[2:], budget_bytes=int(1.5 * one))
    s = torch.cuda.Stream()
    try:
        ra = srv.submit(0, oa, da, rhos[2], mode="mixed", seg_stride=stride)
        srv.wait(ra, 120)
        with torch.cuda.stream(s):
            torch.cuda._sleep(50_000_000)          # tens of ms: the copy runs after it
        res_a = srv.result(ra, stream=s)
        srv.release(ra)
        rb = srv.submit(0, ob, db, rhos[2], mode="mixed", seg_stride=stride)
        srv.wait(rb, 120)
        res_b = srv.result(rb)
        torch.cuda.synchronize()
        srv.release(rb)
        s.synchronize()
    finally:
        srv.close()
    for (o, d), res in (((oa, da), res_a), ((ob, db), res_b)):
        ref = vrt.trace(grids[2], o, d, rhos[2], mode="mixed", segments="stride", seg_stride=stride)
        assert torch.equal(ref["tau"], res["tau"]) and torch.equal(ref["n_seg"], res["n_seg"])
        assert torch.equal(ref["status"], res["status"])


def test_serving_on_grids_with_block_lists(env):
    """Grids built with the block lists of Sect. 2.3 serve like any other:
    every result equals vor_trace on the same grid and on the grid without
    the lists."""
    vrt, torch, ws, grids, rhos = env
    lgrids = [vrt.build_grid(w.sites, w.box, block_lists=True) for w in ws]
    reqs = _requests(ws, 12, seed=13)
    srv = vrt.Server(lgrids, budget_bytes=1 << 30)
    try:
        ids = [srv.submit(r["grid"], r["o"], r["d"], rhos[r["grid"]], mode=r["mode"], seg_stride=24) for r in reqs]
        res = []
        for rid in ids:
            srv.wait(rid, 120)
            res.append(srv.result(rid))
        torch.cuda.synchronize()
        for rid in ids:
            srv.release(rid)
    finally:
        srv.close()
    for r, a in zip(reqs, res):
        for g in (lgrids[r["grid"]], grids[r["grid"]]):
            ref = vrt.trace(g, r["o"], r["d"], rhos[r["grid"]], mode=r["mode"], segments="stride", seg_stride=24)
            assert torch.equal(ref["tau"], a["tau"]) and torch.equal(ref["n_seg"], a["n_seg"])
            assert torch.equal(ref["status"], a["status"])



def test_serving_with_densities_bound_to_the_grids(env):
    """Requests that use the densities bound to their grid
    (VOR_SERVE_GRID_DENSITY), mixed in one server with requests that pass the
    same field as an array: every result is the same bit for bit, and equals
    vor_trace. A request asking for a bound field on a grid without one, or
    passing an array as well, is refused at submission."""
    vrt, torch, ws, _, rhos = env
    bgrids = [vrt.build_grid(w.sites, w.box) for w in ws]
    for g, r in zip(bgrids[:2], rhos[:2]):
        g.bind_density(r)                      # the third grid holds none
    reqs = [r for r in _requests(ws, 30, seed=17) if r["grid"] < 2][:16]
    srv = vrt.Server(bgrids, budget_bytes=1 << 30)
    try:
        ids = []
        for r in reqs:
            ids.append((srv.submit(r["grid"], r["o"], r["d"], None, mode=r["mode"], seg_stride=32,
                                   grid_density=True),
                        srv.submit(r["grid"], r["o"], r["d"], rhos[r["grid"]], mode=r["mode"], seg_stride=32)))
        w = ws[2]
        o = torch.as_tensor(w.sites[:64], device="cuda").contiguous()
        with pytest.raises(vrt.VorError):
            srv.submit(2, o, o, None, mode="mixed", grid_density=True)           # nothing bound
        with pytest.raises(vrt.VorError):
            srv.submit(0, o, o, rhos[0], mode="mixed", grid_density=True)        # both
        res = []
        for a, b in ids:
            srv.wait(a, 120)
            srv.wait(b, 120)
            res.append((srv.result(a), srv.result(b)))
        torch.cuda.synchronize()
        for a, b in ids:
            srv.release(a)
            srv.release(b)
    finally:
        srv.close()
    assert any(float(a["tau"].max()) > 0 for a, _ in res)
    for r, (a, b) in zip(reqs, res):
        assert _same(a, b)
        ref = vrt.trace(bgrids[r["grid"]], r["o"], r["d"], None, mode=r["mode"], segments="stride", seg_stride=32,
                        grid_density=True)
        assert torch.equal(ref["tau"], a["tau"]) and torch.equal(ref["n_seg"], a["n_seg"])
