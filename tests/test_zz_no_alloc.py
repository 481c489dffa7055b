"""vor_trace_noalloc, the trace entry point that allocates nothing (its
control words and start-cell scratch live in a fixed array of the library),
called through the C ABI and checked against vor_trace on the same inputs,
bit for bit: two calls in a row, the second with fewer rays, in another
mode and output layout, so that whatever the first call left in the array
must not reach the second."""
import ctypes

import numpy as np
import pytest

from paper_1310_1854_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vrt():
    import torch
    assert torch.cuda.is_available()
    from paper_1310_1854_amd import vrt as v
    v.load()
    return v


def _call(vrt, name, grid, o, d, rho, out, mode, persistent):
    opts = vrt.TraceOpts(vrt.MODES[mode], 0, 0.0, 1 if persistent else 0, 0, 0, 0, 0.0)
    fn = getattr(vrt.load(), name)
    return fn(grid.handle, vrt._ptr(o), vrt._ptr(d), o.shape[0], vrt._ptr(rho), 1.0, ctypes.byref(opts),
              ctypes.byref(out), vrt._stream())


def _paths(vrt, bufs, n):
    """Every ray's (cells, lengths) from a stride window and its spill chain."""
    stride = bufs.seg_stride
    n_seg = bufs.n_seg.cpu().numpy()
    wc = bufs.seg_cell.cpu().numpy().reshape(n, stride)
    wl = bufs.seg_len.cpu().numpy().reshape(n, stride)
    first = bufs.spill_first.cpu().numpy()
    nxt = bufs.spill_next.cpu().numpy()
    sc = bufs.spill_cell.cpu().numpy()
    sl = bufs.spill_len.cpu().numpy()
    out = []
    for r in range(n):
        k = int(n_seg[r])
        cells, lens = [wc[r, :min(k, stride)]], [wl[r, :min(k, stride)]]
        c, left = int(first[r]), k - stride
        while left > 0:
            assert c >= 0, f"ray {r}: chain ends early"
            m = min(left, vrt.SPILL_CHUNK)
            cells.append(sc[c * vrt.SPILL_CHUNK:c * vrt.SPILL_CHUNK + m])
            lens.append(sl[c * vrt.SPILL_CHUNK:c * vrt.SPILL_CHUNK + m])
            left -= m
            c = int(nxt[c])
        out.append((np.concatenate(cells), np.concatenate(lens)))
    return out


def test_noalloc_equals_vor_trace_twice(vrt):
    import torch
    w = W.exp_disc(M=20_000, N=30_000, seed=91)
    grid = vrt.build_grid(w.sites, w.box)
    o = torch.as_tensor(w.origins, device="cuda").contiguous()
    d = torch.as_tensor(w.dirs, device="cuda").contiguous()
    rho = torch.as_tensor(w.density, device="cuda").contiguous()

    # first call: mixed mode, persistent kernel, exact rows, all 30000 rays
    ref = vrt.TraceBuffers(w.N)
    vrt.trace_into(grid, o, d, rho, ref, mode="mixed", persistent=True)
    off = vrt.exclusive_scan(ref.n_seg)
    total = int(off[-1].item())
    a = vrt.TraceBuffers(w.N, total_segments=total)
    a.ray_off = off
    assert _call(vrt, "vor_trace", grid, o, d, rho, a.struct(), "mixed", True) == vrt.VOR_OK
    b = vrt.TraceBuffers(w.N, total_segments=total, locate_first=False)
    b.ray_off = off
    ob = b.struct()
    ob.work = None
    ob.start_cell = None
    assert _call(vrt, "vor_trace_noalloc", grid, o, d, rho, ob, "mixed", True) == vrt.VOR_OK
    torch.cuda.synchronize()
    for k in ("tau", "n_seg", "status", "n_fallback"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert torch.equal(a.counters[:5], b.counters[:5])   # segments, fallbacks, redecisions, steps, records
    assert torch.equal(a.seg_cell[:total], b.seg_cell[:total]) and torch.equal(a.seg_len[:total], b.seg_len[:total])
    assert int((a.status == 0).sum()) == w.N

    # second call: fewer rays, FP64, one ray per lane, 8-slot windows with spill chains
    n2 = 7000
    o2, d2 = o[:n2].contiguous(), d[:n2].contiguous()
    a2 = vrt.TraceBuffers(n2, seg_stride=8, spill_chunks=4 * n2)
    assert _call(vrt, "vor_trace", grid, o2, d2, rho, a2.struct(), "fp64", False) == vrt.VOR_OK
    b2 = vrt.TraceBuffers(n2, seg_stride=8, spill_chunks=4 * n2, locate_first=False)
    ob2 = b2.struct()
    ob2.work = None
    ob2.start_cell = None
    assert _call(vrt, "vor_trace_noalloc", grid, o2, d2, rho, ob2, "fp64", False) == vrt.VOR_OK
    torch.cuda.synchronize()
    for k in ("tau", "n_seg", "status", "n_fallback"):
        assert torch.equal(getattr(a2, k), getattr(b2, k)), k
    assert int((a2.n_seg > 8).sum()) > 0.5 * n2          # most paths continue in spill chunks
    assert torch.equal(a2.n_seg, ref.n_seg[:n2])          # and they are the first call's paths
    pa, pb = _paths(vrt, a2, n2), _paths(vrt, b2, n2)
    for r in range(n2):
        assert np.array_equal(pa[r][0], pb[r][0]) and np.array_equal(pa[r][1], pb[r][1]), r
    off2 = off[:n2 + 1].cpu().numpy()
    ac, al = a.seg_cell.cpu().numpy(), a.seg_len.cpu().numpy()
    for r in range(0, n2, 97):   # the FP64 paths equal the mixed ones of the first call
        assert np.array_equal(pb[r][0], ac[off2[r]:off2[r + 1]]) and np.array_equal(pb[r][1], al[off2[r]:off2[r + 1]])


def test_noalloc_refuses_what_it_cannot_take(vrt):
    import torch
    w = W.uniform_cube(M=200, N=16, seed=92)
    grid = vrt.build_grid(w.sites, w.box)
    o = torch.as_tensor(w.origins, device="cuda").contiguous()
    d = torch.as_tensor(w.dirs, device="cuda").contiguous()
    bufs = vrt.TraceBuffers(w.N)
    out = bufs.struct()                  # work and start_cell given: the caller's scratch is not taken
    assert _call(vrt, "vor_trace_noalloc", grid, o, d, None, out, "fp64", True) == vrt.VOR_EINVAL
    out.work = None
    out.start_cell = None
    opts = vrt.TraceOpts(0, 0, 0.0, 0, 0, 0, 0, 0.0)
    lib = vrt.load()
    # more rays than the array holds: refused before any device work (the inputs are never read)
    assert lib.vor_trace_noalloc(grid.handle, vrt._ptr(o), vrt._ptr(d), vrt.NOALLOC_MAX_RAYS + 1, None, 1.0,
                                 ctypes.byref(opts), ctypes.byref(out), vrt._stream()) == vrt.VOR_ECAPACITY
    assert _call(vrt, "vor_trace_noalloc", grid, o, d, None, out, "fp64", True) == vrt.VOR_OK
    torch.cuda.synchronize()
    assert int((bufs.status == 0).sum()) == w.N
