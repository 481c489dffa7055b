"""ctypes binding of libvoronoi_rt (include/voronoi_rt.h).

Argument marshalling only: every step runs in the library's HIP kernels.
torch supplies device memory (tensors) and the current HIP stream. torch is
imported before the library is loaded so that both use one HIP runtime.

Names mirror the C ABI: ``build_grid``, ``locate``, ``trace``,
``exclusive_scan``; ``Grid`` owns a ``vor_grid*``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvoronoi_rt.so")

VOR_OK, VOR_EINVAL, VOR_EDUP, VOR_EOUTSIDE, VOR_ENOMEM, VOR_EDEVICE, VOR_ECAPACITY, VOR_EBUDGET, VOR_ETIMEOUT = range(9)
RAY_OK, RAY_OUTSIDE, RAY_BADDIR, RAY_STEPLIMIT, RAY_OVERFLOW = range(5)
MODES = {"fp64": 0, "mixed": 1}
SERVE_GRID_DENSITY = 0x100   # or'ed into a server request's mode: the grid's bound densities

# every symbol include/voronoi_rt.h declares
EXPORTS = ["vor_build_grid", "vor_grid_free", "vor_grid_get_info", "vor_grid_neighbors", "vor_locate",
           "vor_trace", "vor_order_rays", "vor_order_workspace_bytes", "vor_exclusive_scan", "vor_status_str", "vor_version",
           "vor_server_create", "vor_server_submit", "vor_server_poll", "vor_server_wait", "vor_server_result",
           "vor_server_copy_result", "vor_server_release", "vor_server_get_stats", "vor_server_destroy",
           "vor_server_next_done", "vor_grid_truncate_row", "vor_grid_volumes", "vor_grid_bboxes",
           "vor_locate_blocks", "vor_grid_bind_density", "vor_trace_noalloc", "vor_gather_paths"]
NOALLOC_MAX_RAYS = 1 << 22   # VOR_NOALLOC_MAX_RAYS


class VorError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_str(code)} ({code})")


class BuildOpts(ctypes.Structure):
    _fields_ = [("bucket_occupancy", ctypes.c_double), ("block_lists", ctypes.c_int32),
                ("block_occupancy", ctypes.c_double), ("record_layout", ctypes.c_int32)]


RECORD_LAYOUTS = {"auto": 0, "fp32": 1, "compact": 2}


class GridInfo(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int64), ("nnz", ctypes.c_int64), ("nnz_with_walls", ctypes.c_int64),
                ("max_row", ctypes.c_int32), ("dims", ctypes.c_int32 * 3), ("box", ctypes.c_double * 6),
                ("build_ms", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("block_dims", ctypes.c_int32 * 3), ("block_entries", ctypes.c_int64),
                ("record_layout", ctypes.c_int32)]


class TraceOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_steps", ctypes.c_int32), ("eps_mix", ctypes.c_double),
                ("persistent", ctypes.c_int32), ("start_given", ctypes.c_int32), ("enter", ctypes.c_int32),
                ("grid_density", ctypes.c_int32), ("eps_fb", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """vor_allocator: device memory for a grid's arrays."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


def torch_allocator() -> Allocator:
    """A vor_allocator over torch's caching allocator: the grid's arrays come
    from (and go back to) the same pool as torch's tensors. Keep the returned
    object alive as long as any grid built with it (Grid does)."""
    def _alloc(nbytes, ctx, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except RuntimeError:   # out of memory: the library reports VOR_ENOMEM
            return None

    def _free(ptr, nbytes, ctx, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    a._keep = (_alloc, _free)
    return a


class TraceOut(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_void_p), ("n_seg", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("n_fallback", ctypes.c_void_p), ("seg_cell", ctypes.c_void_p), ("seg_len", ctypes.c_void_p),
                ("seg_stride", ctypes.c_int64), ("ray_off", ctypes.c_void_p), ("counters", ctypes.c_void_p),
                ("work", ctypes.c_void_p), ("spill_first", ctypes.c_void_p), ("spill_next", ctypes.c_void_p),
                ("spill_cell", ctypes.c_void_p), ("spill_len", ctypes.c_void_p), ("spill_chunks", ctypes.c_int64),
                ("ray_order", ctypes.c_void_p), ("start_cell", ctypes.c_void_p),
                ("tau_stop", ctypes.c_void_p), ("stop_cell", ctypes.c_void_p), ("stop_s", ctypes.c_void_p),
                ("tally_len", ctypes.c_void_p), ("tally_abs", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


SPILL_CHUNK = 64     # VOR_SPILL_CHUNK
WORK_WORDS = 16      # VOR_WORK_WORDS


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("crossings", ctypes.c_int64), ("fp64_redecisions", ctypes.c_int64),
                ("fallbacks", ctypes.c_int64), ("launches", ctypes.c_int64), ("running", ctypes.c_int64),
                ("waiting", ctypes.c_int64),
                ("budget_bytes", ctypes.c_int64), ("used_bytes", ctypes.c_int64), ("uptime_s", ctypes.c_double),
                ("reruns", ctypes.c_int64)]


_lib = None


def load(path: str = None):
    """Load the HIP library (the in-tree build unless VRT_LIB names another
    build of the same sources); raises if it has not been built (there is no
    CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("VRT_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libvoronoi_rt.so not built at {path}; run paper_1310_1854_amd.build_lib")
    lib = ctypes.CDLL(path)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.vor_build_grid.argtypes = [P, I64, P, P, P, P, ctypes.POINTER(P)]
    lib.vor_build_grid.restype = ctypes.c_int
    lib.vor_grid_free.argtypes = [P]
    lib.vor_grid_free.restype = None
    lib.vor_grid_get_info.argtypes = [P, ctypes.POINTER(GridInfo)]
    lib.vor_grid_get_info.restype = ctypes.c_int
    lib.vor_grid_volumes.argtypes = [P, P, P]
    lib.vor_grid_volumes.restype = ctypes.c_int
    lib.vor_grid_bind_density.argtypes = [P, P, P]
    lib.vor_grid_bind_density.restype = ctypes.c_int
    lib.vor_grid_truncate_row.argtypes = [P, I64, I32]
    lib.vor_grid_truncate_row.restype = ctypes.c_int
    lib.vor_grid_neighbors.argtypes = [P, P, P, P]
    lib.vor_grid_neighbors.restype = ctypes.c_int
    lib.vor_locate.argtypes = [P, P, I64, P, P]
    lib.vor_locate.restype = ctypes.c_int
    lib.vor_locate_blocks.argtypes = [P, P, I64, P, P]
    lib.vor_locate_blocks.restype = ctypes.c_int
    lib.vor_grid_bboxes.argtypes = [P, P, P]
    lib.vor_grid_bboxes.restype = ctypes.c_int
    lib.vor_trace.argtypes = [P, P, P, I64, P, D, ctypes.POINTER(TraceOpts), ctypes.POINTER(TraceOut), P]
    lib.vor_trace.restype = ctypes.c_int
    lib.vor_trace_noalloc.argtypes = [P, P, P, I64, P, D, ctypes.POINTER(TraceOpts), ctypes.POINTER(TraceOut), P]
    lib.vor_trace_noalloc.restype = ctypes.c_int
    lib.vor_order_rays.argtypes = [P, P, P, I64, P, P, I64, P]
    lib.vor_order_rays.restype = ctypes.c_int
    lib.vor_order_workspace_bytes.argtypes = [I64]
    lib.vor_order_workspace_bytes.restype = ctypes.c_int64
    lib.vor_exclusive_scan.argtypes = [P, I64, P, P]
    lib.vor_exclusive_scan.restype = ctypes.c_int
    lib.vor_gather_paths.argtypes = [P, I64, P, P, I64, P, P, P, P, P, P, P, P]
    lib.vor_gather_paths.restype = ctypes.c_int
    lib.vor_status_str.argtypes = [ctypes.c_int]
    lib.vor_status_str.restype = ctypes.c_char_p
    lib.vor_version.argtypes = []
    lib.vor_version.restype = ctypes.c_char_p
    lib.vor_server_create.argtypes = [ctypes.POINTER(P), I32, I64, ctypes.POINTER(P)]
    lib.vor_server_create.restype = ctypes.c_int
    lib.vor_server_submit.argtypes = [P, I32, P, P, I64, P, D, I32, I64, I64, P, ctypes.POINTER(I64)]
    lib.vor_server_submit.restype = ctypes.c_int
    lib.vor_server_poll.argtypes = [P, I64, ctypes.POINTER(I32)]
    lib.vor_server_poll.restype = ctypes.c_int
    lib.vor_server_wait.argtypes = [P, I64, D]
    lib.vor_server_wait.restype = ctypes.c_int
    lib.vor_server_next_done.argtypes = [P, D, ctypes.POINTER(I64)]
    lib.vor_server_next_done.restype = ctypes.c_int
    lib.vor_server_result.argtypes = [P, I64, ctypes.POINTER(TraceOut), ctypes.POINTER(D)]
    lib.vor_server_result.restype = ctypes.c_int
    lib.vor_server_copy_result.argtypes = [P, I64, P, P, P, P, P, P, P]
    lib.vor_server_copy_result.restype = ctypes.c_int
    lib.vor_server_release.argtypes = [P, I64]
    lib.vor_server_release.restype = ctypes.c_int
    lib.vor_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.vor_server_get_stats.restype = ctypes.c_int
    lib.vor_server_destroy.argtypes = [P]
    lib.vor_server_destroy.restype = None
    _lib = lib
    return lib


def status_str(code: int) -> str:
    return load().vor_status_str(int(code)).decode()


def _check(code: int, what: str):
    if code != VOR_OK:
        raise VorError(code, what)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f64(x, shape_last=None, device=None) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64, device=device or "cuda")
    t = t.contiguous()
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"expected an (N, {shape_last}) array")
    return t


class Grid:
    """A built grid (owns the library's vor_grid)."""

    def __init__(self, handle: int, M: int, box, allocator: Optional[Allocator] = None):
        self._h = ctypes.c_void_p(handle)
        self.M = M
        self.box = [float(b) for b in box]
        self._allocator = allocator   # its callbacks must outlive the grid

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = GridInfo()
        _check(load().vor_grid_get_info(self._h, ctypes.byref(inf)), "vor_grid_get_info")
        return dict(n_sites=inf.n_sites, nnz=inf.nnz, nnz_with_walls=inf.nnz_with_walls, max_row=inf.max_row,
                    dims=list(inf.dims), box=list(inf.box), build_ms=inf.build_ms, device_bytes=inf.device_bytes,
                    block_dims=list(inf.block_dims), block_entries=inf.block_entries,
                    record_layout={1: "fp32", 2: "compact"}.get(inf.record_layout, inf.record_layout))

    def neighbors(self, stream=None):
        """(row_ptr int64[M+1], col int32[nnz]) in user order, walls as -1..-6."""
        inf = self.info()
        row_ptr = torch.empty(self.M + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(max(inf["nnz_with_walls"], 1), dtype=torch.int32, device="cuda")
        _check(load().vor_grid_neighbors(self._h, _ptr(row_ptr), _ptr(col), _stream(stream)), "vor_grid_neighbors")
        return row_ptr, col[: inf["nnz_with_walls"]]

    def volumes(self, stream=None) -> torch.Tensor:
        """Volume of every cell (user order), from the builder's clipped cells."""
        out = torch.empty(self.M, dtype=torch.float64, device="cuda")
        _check(load().vor_grid_volumes(self.handle, _ptr(out), _stream(stream)), "vor_grid_volumes")
        return out

    def bboxes(self, stream=None) -> torch.Tensor:
        """Bounding box of every cell (user order, M x 6: min xyz, max xyz);
        needs a grid built with block_lists=True."""
        out = torch.empty((self.M, 6), dtype=torch.float64, device="cuda")
        _check(load().vor_grid_bboxes(self.handle, _ptr(out), _stream(stream)), "vor_grid_bboxes")
        return out

    def bind_density(self, density: Optional[torch.Tensor], stream=None) -> None:
        """vor_grid_bind_density: keep a copy of ``density`` (float64, one value
        per site, user order) in the grid for traces with grid_density=True;
        None removes it."""
        if density is not None and (density.dtype != torch.float64 or not density.is_cuda
                                    or not density.is_contiguous() or density.numel() != self.M):
            raise ValueError("density must be a contiguous float64 CUDA tensor with one value per site")
        _check(load().vor_grid_bind_density(self.handle, _ptr(density), _stream(stream)), "vor_grid_bind_density")

    def truncate_row(self, site: int, keep: int) -> None:
        """Diagnostic (vor_grid_truncate_row): drop faces of one cell from the
        neighbour table, to exercise the no-exit fallback."""
        _check(load().vor_grid_truncate_row(self.handle, int(site), int(keep)), "vor_grid_truncate_row")

    def free(self):
        if self._h is not None and self._h.value:
            load().vor_grid_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def build_grid(sites, box: Sequence[float], bucket_occupancy: float = 0.0, block_lists: bool = False,
               block_occupancy: float = 0.0, allocator: Optional[Allocator] = None, stream=None,
               records: str = "auto") -> Grid:
    """vor_build_grid; block_lists also builds the block-list locate
    structure (vor_locate_blocks) and keeps the cells' bounding boxes;
    allocator (e.g. torch_allocator()): where the grid's device memory
    comes from (default hipMalloc); records: the layout of the records
    mixed-mode traces read ("auto", "fp32" or "compact"; same results)."""
    if records not in RECORD_LAYOUTS:
        raise ValueError(f"records must be one of {sorted(RECORD_LAYOUTS)}")
    sites_d = _dev_f64(sites, 3)
    box_h = (ctypes.c_double * 6)(*[float(b) for b in box])
    opts = BuildOpts(float(bucket_occupancy), 1 if block_lists else 0, float(block_occupancy),
                     RECORD_LAYOUTS[records])
    h = ctypes.c_void_p()
    _check(load().vor_build_grid(_ptr(sites_d), sites_d.shape[0], box_h, ctypes.byref(opts),
                                 None if allocator is None else ctypes.byref(allocator), _stream(stream),
                                 ctypes.byref(h)), "vor_build_grid")
    return Grid(h.value, sites_d.shape[0], box, allocator)


def locate(grid: Grid, pts, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    p = _dev_f64(pts, 3)
    n = p.shape[0]
    cell = out if out is not None else torch.empty(n, dtype=torch.int32, device="cuda")
    _check(load().vor_locate(grid.handle, _ptr(p), n, _ptr(cell), _stream(stream)), "vor_locate")
    return cell


def locate_blocks(grid: Grid, pts, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """vor_locate_blocks: C(r) through the block lists of Sect. 2.3."""
    p = _dev_f64(pts, 3)
    n = p.shape[0]
    cell = out if out is not None else torch.empty(n, dtype=torch.int32, device="cuda")
    _check(load().vor_locate_blocks(grid.handle, _ptr(p), n, _ptr(cell), _stream(stream)), "vor_locate_blocks")
    return cell


def exclusive_scan(counts: torch.Tensor, stream=None) -> torch.Tensor:
    c = counts.to(dtype=torch.int32).contiguous()
    off = torch.empty(c.numel() + 1, dtype=torch.int64, device=c.device)
    _check(load().vor_exclusive_scan(_ptr(c), c.numel(), _ptr(off), _stream(stream)), "vor_exclusive_scan")
    return off


COUNTERS = ["segments", "fallbacks", "fp64_redecisions", "steps", "records", "r5", "r6", "r7"]


class TraceBuffers:
    """Preallocated outputs of ``trace`` for N rays (reused across calls).

    seg_stride > 0: a window of seg_stride slots per ray; with spill_chunks
    > 0 longer paths continue in chained spill chunks of SPILL_CHUNK slots.
    total_segments > 0 (and seg_stride 0): exact CSR windows from ray_off.
    ordered: also hold a processing order (vor_order_rays) and its workspace."""

    def __init__(self, N: int, seg_stride: int = 0, total_segments: int = 0, spill_chunks: int = 0,
                 device="cuda", counters=True, ordered=False, locate_first=True, stops=False):
        self.N = N
        # interaction points (vor_trace_out.stop_cell / stop_s), filled when a trace is given tau_stop
        self.stop_cell = torch.empty(max(N, 1), dtype=torch.int32, device=device) if stops else None
        self.stop_s = torch.empty(max(N, 1), dtype=torch.float64, device=device) if stops else None
        # scratch for the start-cell pass (vor_trace_out.start_cell)
        self.start_cell = torch.empty(max(N, 1), dtype=torch.int32, device=device) if locate_first else None
        self.tau = torch.empty(N, dtype=torch.float64, device=device)
        self.n_seg = torch.empty(N, dtype=torch.int32, device=device)
        self.status = torch.empty(N, dtype=torch.uint8, device=device)
        self.n_fallback = torch.empty(N, dtype=torch.int32, device=device)
        self.seg_stride = int(seg_stride)
        nslots = N * self.seg_stride if self.seg_stride > 0 else int(total_segments)
        want_segs = self.seg_stride > 0 or total_segments > 0
        self.seg_cell = torch.empty(max(nslots, 1), dtype=torch.int32, device=device) if want_segs else None
        self.seg_len = torch.empty(max(nslots, 1), dtype=torch.float64, device=device) if want_segs else None
        self.ray_off: Optional[torch.Tensor] = None
        self.counters = torch.zeros(8, dtype=torch.int64, device=device) if counters else None
        self.work = torch.zeros(WORK_WORDS, dtype=torch.int64, device=device)
        self.spill_chunks = int(spill_chunks) if self.seg_stride > 0 else 0
        if self.spill_chunks > 0:
            self.spill_first = torch.empty(N, dtype=torch.int64, device=device)
            self.spill_next = torch.empty(self.spill_chunks, dtype=torch.int32, device=device)
            self.spill_cell = torch.empty(self.spill_chunks * SPILL_CHUNK, dtype=torch.int32, device=device)
            self.spill_len = torch.empty(self.spill_chunks * SPILL_CHUNK, dtype=torch.float64, device=device)
        else:
            self.spill_first = self.spill_next = self.spill_cell = self.spill_len = None
        self.order = None
        self.order_ws = None
        if ordered:
            self.order = torch.empty(max(N, 1), dtype=torch.int32, device=device)
            self.order_ws = torch.empty(int(load().vor_order_workspace_bytes(N)), dtype=torch.uint8, device=device)

    def struct(self, use_order: bool = False, tau_stop=None, tally_len=None, tally_abs=None,
               weight=None) -> TraceOut:
        o = TraceOut()
        if tau_stop is not None:
            if self.stop_cell is None:
                raise ValueError("buffers were made without stops=True")
            o.tau_stop = tau_stop.data_ptr()
            o.stop_cell = self.stop_cell.data_ptr()
            o.stop_s = self.stop_s.data_ptr()
        o.tally_len = tally_len.data_ptr() if tally_len is not None else None
        o.tally_abs = tally_abs.data_ptr() if tally_abs is not None else None
        o.weight = weight.data_ptr() if weight is not None else None
        o.tau = self.tau.data_ptr()
        o.n_seg = self.n_seg.data_ptr()
        o.status = self.status.data_ptr()
        o.n_fallback = self.n_fallback.data_ptr()
        o.seg_cell = self.seg_cell.data_ptr() if self.seg_cell is not None else None
        o.seg_len = self.seg_len.data_ptr() if self.seg_len is not None else None
        o.seg_stride = self.seg_stride if self.seg_cell is not None else 0
        o.ray_off = self.ray_off.data_ptr() if self.ray_off is not None else None
        o.counters = self.counters.data_ptr() if self.counters is not None else None
        o.work = self.work.data_ptr()
        if self.spill_chunks > 0:
            o.spill_first = self.spill_first.data_ptr()
            o.spill_next = self.spill_next.data_ptr()
            o.spill_cell = self.spill_cell.data_ptr()
            o.spill_len = self.spill_len.data_ptr()
            o.spill_chunks = self.spill_chunks
        if use_order and self.order is not None:
            o.ray_order = self.order.data_ptr()
        if self.start_cell is not None:
            o.start_cell = self.start_cell.data_ptr()
        return o


def order_rays(grid: Grid, origins: torch.Tensor, dirs: torch.Tensor, order: torch.Tensor,
               workspace: torch.Tensor, stream=None) -> None:
    """Enqueue vor_order_rays into ``order`` (int32, N)."""
    n = origins.shape[0]
    _check(load().vor_order_rays(grid.handle, _ptr(origins), _ptr(dirs), n, _ptr(order), _ptr(workspace),
                                 workspace.numel(), _stream(stream)), "vor_order_rays")


def n_rays(origins) -> int:
    return int(origins.shape[0])


def _check_density(density: Optional[torch.Tensor], grid: "Grid") -> None:
    if density is not None and (density.dtype != torch.float64 or not density.is_cuda
                                or not density.is_contiguous() or density.numel() != grid.M):
        raise ValueError("density must be a contiguous float64 device tensor with one value per site")


def trace_into(grid: Grid, origins: torch.Tensor, dirs: torch.Tensor, density: Optional[torch.Tensor],
               bufs: TraceBuffers, kappa: float = 1.0, mode: str = "fp64", max_steps: int = 0,
               eps_mix: float = 0.0, persistent: bool = False, ordered: bool = False, start_given: bool = False,
               tau_stop: Optional[torch.Tensor] = None, tally_len: Optional[torch.Tensor] = None,
               tally_abs: Optional[torch.Tensor] = None, weight: Optional[torch.Tensor] = None,
               enter: bool = False, grid_density: bool = False, eps_fb: float = 0.0, stream=None) -> None:
    """Enqueue one vor_trace into preallocated buffers (no allocation, no
    sync); with ``ordered`` the rays are first put in coherent order by
    vor_order_rays (buffers made with ordered=True). ``start_given``: the
    buffers' start cells are those of an earlier call on the same rays.
    ``tau_stop`` (float64 [N], buffers made with stops=True): interaction
    points; ``tally_len`` / ``tally_abs`` (float64 [M], accumulated) and
    ``weight`` (float64 [N]): per-cell tallies. ``grid_density``: the
    densities bound with Grid.bind_density (``density`` must be None)."""
    for name, t, size in (("tau_stop", tau_stop, n_rays(origins)), ("weight", weight, n_rays(origins)),
                          ("tally_len", tally_len, grid.M), ("tally_abs", tally_abs, grid.M)):
        if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
                              or t.numel() != size):
            raise ValueError(f"{name} must be a contiguous float64 device tensor of {size} values")
    n = origins.shape[0]
    if origins.dtype != torch.float64 or dirs.dtype != torch.float64 or not origins.is_contiguous() \
            or not dirs.is_contiguous() or origins.shape != dirs.shape or n != bufs.N:
        raise ValueError("origins/dirs must be contiguous float64 (N, 3) tensors matching the buffers")
    if not origins.is_cuda or not dirs.is_cuda:
        raise ValueError("origins/dirs must be device tensors")
    _check_density(density, grid)
    if ordered:
        if bufs.order is None:
            raise ValueError("buffers were made without ordered=True")
        if not start_given:   # the start cells were located in the earlier call's order
            order_rays(grid, origins, dirs, bufs.order, bufs.order_ws, stream=stream)
    if start_given and bufs.start_cell is None:
        raise ValueError("start_given needs buffers made with locate_first=True")
    opts = TraceOpts(MODES[mode], int(max_steps), float(eps_mix), 1 if persistent else 0, 1 if start_given else 0,
                     1 if enter else 0, 1 if grid_density else 0, float(eps_fb))
    out = bufs.struct(use_order=ordered, tau_stop=tau_stop, tally_len=tally_len, tally_abs=tally_abs,
                      weight=weight)
    _check(load().vor_trace(grid.handle, _ptr(origins), _ptr(dirs), n, _ptr(density), float(kappa),
                            ctypes.byref(opts), ctypes.byref(out), _stream(stream)), "vor_trace")


def trace(grid: Grid, origins, dirs, density=None, kappa: float = 1.0, mode: str = "fp64",
          segments: str = "exact", seg_stride: int = 64, spill_chunks: int = 0, max_steps: int = 0,
          eps_mix: float = 0.0, persistent: bool = False, ordered: bool = False, locate_first: bool = True,
          tau_stop=None, weight=None, tallies: bool = False, enter: bool = False, grid_density: bool = False,
          eps_fb: float = 0.0, stream=None) -> dict:
    """Paths of N rays. ``segments``: "none" (tau only), "stride" (a window
    of ``seg_stride`` slots per ray; longer paths continue in up to
    ``spill_chunks`` chained spill chunks, or report RAY_OVERFLOW), "exact"
    (every path whole in compact rows: one traversal into windows of
    ``seg_stride`` slots and a spill sized from ``spill_chunks``, traced
    again with the spill it asked for if that was too small, then a scan
    and vor_gather_paths; with ``tallies`` the two-pass route, so that no
    tally is deposited twice), or "exact_two_pass" (a tau-only counting
    pass, a scan, then a pass that writes every segment at its offset). ``locate_first``: start cells in a pass of
    their own (vor_trace_out.start_cell) rather than at each ray's start.
    ``tau_stop``: interaction points (stop_cell, stop_s); ``tallies``: the
    per-cell tallies tally_len and tally_abs (with ``weight``); ``enter``:
    rays from outside the box start where they enter it; ``grid_density``:
    the densities bound with Grid.bind_density; ``eps_fb``: the no-exit
    fallback's advance (0: 1e-12 of the box diagonal). Returns a dict of
    device tensors."""
    o = _dev_f64(origins, 3)
    d = _dev_f64(dirs, 3)
    rho = None if density is None else _dev_f64(density).reshape(-1)
    n = o.shape[0]
    ts = None if tau_stop is None else _dev_f64(tau_stop).reshape(-1)
    wt = None if weight is None else _dev_f64(weight).reshape(-1)
    t_len = torch.zeros(grid.M, dtype=torch.float64, device="cuda") if tallies else None
    t_abs = torch.zeros(grid.M, dtype=torch.float64, device="cuda") if tallies else None
    kw = dict(kappa=kappa, mode=mode, max_steps=max_steps, eps_mix=eps_mix, persistent=persistent, ordered=ordered,
              stream=stream, tau_stop=ts, weight=wt, tally_len=t_len, tally_abs=t_abs, enter=enter,
              grid_density=grid_density, eps_fb=eps_fb)
    lf = dict(ordered=ordered, locate_first=locate_first, stops=ts is not None)
    if segments == "none":
        b = TraceBuffers(n, **lf)
        trace_into(grid, o, d, rho, b, **kw)
    elif segments == "stride":
        b = TraceBuffers(n, seg_stride=seg_stride, spill_chunks=spill_chunks, **lf)
        trace_into(grid, o, d, rho, b, **kw)
    elif segments == "exact" and not tallies:
        chunks = spill_chunks if spill_chunks > 0 else n // 8 + 1
        while True:
            w = TraceBuffers(n, seg_stride=seg_stride, spill_chunks=chunks, **lf)
            trace_into(grid, o, d, rho, w, **kw)
            asked = int(w.work[1].item())
            if asked <= chunks:
                break
            chunks = asked
            del w
        off = exclusive_scan(w.n_seg, stream=stream)
        total = int(off[-1].item())
        b = TraceBuffers(n, total_segments=max(total, 1), ordered=False, locate_first=False, counters=False)
        b.tau, b.n_seg, b.status, b.n_fallback, b.counters, b.work = w.tau, w.n_seg, w.status, w.n_fallback, \
            w.counters, w.work
        b.stop_cell, b.stop_s = w.stop_cell, w.stop_s
        b.ray_off = off
        gather_paths(w, off, b.seg_cell, b.seg_len, stream=stream)
    elif segments in ("exact", "exact_two_pass"):
        b0 = TraceBuffers(n, **lf)
        trace_into(grid, o, d, rho, b0, **dict(kw, tally_len=None, tally_abs=None, weight=None))   # counting pass
        off = exclusive_scan(b0.n_seg, stream=stream)
        total = int(off[-1].item())
        b = TraceBuffers(n, total_segments=max(total, 1), **lf)
        b.ray_off = off
        trace_into(grid, o, d, rho, b, **kw)
    else:
        raise ValueError("segments must be none, stride, exact or exact_two_pass")
    res = dict(tau=b.tau, n_seg=b.n_seg, status=b.status, n_fallback=b.n_fallback, counters=b.counters, work=b.work)
    if ts is not None:
        res.update(stop_cell=b.stop_cell, stop_s=b.stop_s)
    if tallies:
        res.update(tally_len=t_len, tally_abs=t_abs)
    if b.seg_cell is not None:
        res.update(seg_cell=b.seg_cell, seg_len=b.seg_len)
        res["ray_off"] = b.ray_off if b.ray_off is not None else \
            torch.arange(0, (n + 1) * b.seg_stride, b.seg_stride, dtype=torch.int64, device="cuda")
        res["seg_stride"] = b.seg_stride
        if b.spill_chunks > 0:
            res.update(spill_first=b.spill_first, spill_next=b.spill_next, spill_cell=b.spill_cell,
                       spill_len=b.spill_len)
    return res


def gather_paths(bufs: "TraceBuffers", ray_off: torch.Tensor, seg_cell: torch.Tensor, seg_len: torch.Tensor,
                 stream=None) -> None:
    """vor_gather_paths: the whole paths of a trace into segment windows
    (``bufs``, seg_stride > 0) as compact rows at ``ray_off`` (the exclusive
    scan of bufs.n_seg)."""
    if bufs.seg_stride <= 0 or bufs.seg_cell is None:
        raise ValueError("gather_paths needs the buffers of a trace with segment windows")
    n = bufs.N
    if ray_off.dtype != torch.int64 or ray_off.numel() != n + 1 or not ray_off.is_cuda:
        raise ValueError("ray_off must be a device int64 tensor of N + 1 offsets")
    for t, dt in ((seg_cell, torch.int32), (seg_len, torch.float64)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError("seg_cell / seg_len must be contiguous int32 / float64 device tensors")
    sp = bufs.spill_chunks > 0
    _check(load().vor_gather_paths(_ptr(bufs.n_seg), n, _ptr(bufs.seg_cell), _ptr(bufs.seg_len), bufs.seg_stride,
                                   _ptr(bufs.spill_first) if sp else None, _ptr(bufs.spill_next) if sp else None,
                                   _ptr(bufs.spill_cell) if sp else None, _ptr(bufs.spill_len) if sp else None,
                                   _ptr(ray_off), _ptr(seg_cell), _ptr(seg_len), _stream(stream)),
           "vor_gather_paths")


def ray_path(res: dict, r: int, host: Optional[dict] = None):
    """(cells, lengths) of ray r of a trace result, from its window and its
    spill chain. ``host`` caches numpy copies of the spill arrays."""
    n = int(res["n_seg"][r])
    stride = res.get("seg_stride", 0)
    o = int(res["ray_off"][r])
    if stride <= 0 or n <= stride:
        return res["seg_cell"][o:o + n].cpu().numpy(), res["seg_len"][o:o + n].cpu().numpy()
    if "spill_first" not in res:
        raise ValueError(f"ray {r}: path past its window was not stored")
    if host is None:
        host = {}
    if "next" not in host:
        host["first"] = res["spill_first"].cpu().numpy()
        host["next"] = res["spill_next"].cpu().numpy()
    cells = [res["seg_cell"][o:o + stride].cpu().numpy()]
    lens = [res["seg_len"][o:o + stride].cpu().numpy()]
    c = int(host["first"][r])
    left = n - stride
    while left > 0:
        if c < 0:
            raise ValueError(f"ray {r}: spill chain ends early")
        k = min(left, SPILL_CHUNK)
        cells.append(res["spill_cell"][c * SPILL_CHUNK:c * SPILL_CHUNK + k].cpu().numpy())
        lens.append(res["spill_len"][c * SPILL_CHUNK:c * SPILL_CHUNK + k].cpu().numpy())
        left -= k
        c = int(host["next"][c])
    return np.concatenate(cells), np.concatenate(lens)


class Server:
    """A continuous-batching path server over resident grids (vor_server_*).
    Input tensors of a request are kept alive here until it is released."""

    def __init__(self, grids, budget_bytes: int):
        self.grids = list(grids)
        arr = (ctypes.c_void_p * len(self.grids))(*[g.handle.value for g in self.grids])
        h = ctypes.c_void_p()
        _check(load().vor_server_create(arr, len(self.grids), int(budget_bytes), ctypes.byref(h)),
               "vor_server_create")
        self._h = h
        self._keep = {}

    def submit(self, grid: int, origins: torch.Tensor, dirs: torch.Tensor, density: Optional[torch.Tensor] = None,
               kappa: float = 1.0, mode: str = "fp64", seg_stride: int = 0, spill_chunks: Optional[int] = None,
               grid_density: bool = False, stream=None) -> int:
        """Queue a request; ``grid_density``: use the densities bound to the
        grid (Grid.bind_density) instead of ``density``, which must be None.
        ``spill_chunks``: the first pool of spill chunks for segments past
        the windows (None: one chunk per 8 rays); a pool too small only
        costs a second run of the request. The request waits for the work
        already enqueued on ``stream`` (default: the current stream)."""
        if origins.dtype != torch.float64 or dirs.dtype != torch.float64 or not origins.is_contiguous() \
                or not dirs.is_contiguous() or origins.dim() != 2 or origins.shape[1] != 3 \
                or origins.shape != dirs.shape or not origins.is_cuda or not dirs.is_cuda:
            raise ValueError("origins/dirs must be contiguous float64 (N, 3) device tensors")
        if 0 <= grid < len(self.grids):   # (a grid that does not exist is the library's VOR_EINVAL)
            _check_density(density, self.grids[grid])
        n = origins.shape[0]
        stride = int(seg_stride)
        chunks = 0 if stride <= 0 else (n // 8 + 1 if spill_chunks is None else int(spill_chunks))
        rid = ctypes.c_int64()
        m = MODES[mode] | (SERVE_GRID_DENSITY if grid_density else 0)
        _check(load().vor_server_submit(self._h, int(grid), _ptr(origins), _ptr(dirs), n, _ptr(density),
                                        float(kappa), m, stride, chunks, _stream(stream), ctypes.byref(rid)),
               "vor_server_submit")
        self._keep[rid.value] = (origins, dirs, density, stride, n)
        return rid.value

    def poll(self, req: int) -> bool:
        d = ctypes.c_int32()
        _check(load().vor_server_poll(self._h, req, ctypes.byref(d)), "vor_server_poll")
        return bool(d.value)

    def wait(self, req: int, timeout_s: float = 60.0) -> None:
        _check(load().vor_server_wait(self._h, req, float(timeout_s)), "vor_server_wait")

    def next_done(self, timeout_s: float = 60.0) -> Optional[int]:
        """The next request to complete (completion order), or None when none
        completes within timeout_s."""
        rid = ctypes.c_int64()
        code = load().vor_server_next_done(self._h, float(timeout_s), ctypes.byref(rid))
        if code == VOR_ETIMEOUT:
            return None
        _check(code, "vor_server_next_done")
        return rid.value

    def latency(self, req: int) -> float:
        o = TraceOut()
        lat = ctypes.c_double()
        _check(load().vor_server_result(self._h, req, ctypes.byref(o), ctypes.byref(lat)), "vor_server_result")
        return lat.value

    def result(self, req: int, stream=None, paths: bool = True) -> dict:
        """Copy the request's outputs into new tensors: tau, n_seg, status
        and, for a request with segments (unless ``paths`` is False), its
        whole paths as compact rows (ray_off, seg_cell, seg_len: ray i's
        segments at [ray_off[i], ray_off[i + 1]))."""
        _, _, _, stride, n = self._keep[req]
        res = dict(tau=torch.empty(n, dtype=torch.float64, device="cuda"),
                   n_seg=torch.empty(n, dtype=torch.int32, device="cuda"),
                   status=torch.empty(n, dtype=torch.uint8, device="cuda"))
        lib = load()
        if stride > 0 and paths:
            _check(lib.vor_server_copy_result(self._h, req, None, _ptr(res["n_seg"]), None, None, None, None,
                                              _stream(stream)), "vor_server_copy_result")
            off = exclusive_scan(res["n_seg"], stream=stream)
            (stream if stream is not None else torch.cuda.current_stream()).synchronize()   # the total is read here
            total = int(off[-1].item())
            res["ray_off"] = off
            res["seg_cell"] = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
            res["seg_len"] = torch.empty(max(total, 1), dtype=torch.float64, device="cuda")
        _check(lib.vor_server_copy_result(self._h, req, _ptr(res["tau"]), _ptr(res["n_seg"]), _ptr(res["status"]),
                                          _ptr(res.get("ray_off")), _ptr(res.get("seg_cell")),
                                          _ptr(res.get("seg_len")), _stream(stream)), "vor_server_copy_result")
        res["seg_stride"] = stride
        return res

    def release(self, req: int) -> None:
        _check(load().vor_server_release(self._h, req), "vor_server_release")
        self._keep.pop(req, None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().vor_server_get_stats(self._h, ctypes.byref(st)), "vor_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            load().vor_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def version() -> str:
    return load().vor_version().decode()
