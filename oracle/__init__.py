"""Test oracle for straight paths through a box-clipped 3D Voronoi grid.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this package; the product library never does, and this
package imports nothing from it.

Three independent CPU implementations of the path definition live here,
and beside them a baseline for timing only:

* ``oracle.c`` (loaded through ctypes): FP64 brute force over all sites --
  nearest-site location, paths with optical depth and near-tie flags, and
  cell faces / volumes by clipping candidate face planes.
* ``exact.py``: exact rational paths by a sweep over all pairwise bisector
  crossings (tiny inputs only).
* ``dda.py``: closed-form paths through tensor-product lattices, whose
  Voronoi cells are cuboids.
* ``nbtrace.c`` (baseline, not an oracle): the paper's own neighbour-list
  path loop in FP64 on the CPU, on one or several cores, timed beside the
  GPU for the comparison with the paper's single-core timing; checked
  against the oracle in tests/test_nbtrace.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ST_OK, ST_OUTSIDE, ST_BADDIR, ST_STEPLIMIT, ST_OVERFLOW = 0, 1, 2, 3, 4
WALLS = {-1: "xmin", -2: "xmax", -3: "ymin", -4: "ymax", -5: "zmin", -6: "zmax"}
ETA = 1e-9   # near-tie threshold, relative to the chord length

_lib = None


def compile_oracle(src: str, out: str) -> str:
    """gcc -O2, OpenMP, no fast-math and no FMA contraction (plain IEEE FP64)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", src, "-o", out + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


_NB_SRC = os.path.join(_HERE, "nbtrace.c")
_NB_LIB = os.path.join(_HERE, "libnbtrace.so")
_nblib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (and the nbtrace.c baseline)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_oracle(_SRC, _LIB)
    if force or not os.path.exists(_NB_LIB) or os.path.getmtime(_NB_LIB) < os.path.getmtime(_NB_SRC):
        compile_oracle(_NB_SRC, _NB_LIB)
    return _LIB


def nbtrace(sites, box, row_ptr, col, density, origins, dirs, start, kappa=1.0, threads=0):
    """The paper's neighbour-list path loop on the CPU (nbtrace.c): per-ray
    segment counts, tau and no-exit events. row_ptr/col: neighbour lists
    (walls -1..-6); start: the start cell of every ray (< 0: no path)."""
    global _nblib
    if _nblib is None:
        if not os.path.exists(_NB_LIB) or os.path.getmtime(_NB_LIB) < os.path.getmtime(_NB_SRC):
            compile_oracle(_NB_SRC, _NB_LIB)
        lib = ctypes.CDLL(_NB_LIB)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        lib.nbtrace_paths.argtypes = [P, I64, P, P, P, P, ctypes.c_double, P, P, P, I64, ctypes.c_int, P, P, P]
        lib.nbtrace_paths.restype = ctypes.c_int
        _nblib = lib
    sites = _f64(sites, (-1, 3))
    box = _f64(box, (6,))
    origins = _f64(origins, (-1, 3))
    dirs = _f64(dirs, (-1, 3))
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    st = np.ascontiguousarray(start, dtype=np.int32)
    rho = None if density is None else _f64(density, (-1,))
    N = origins.shape[0]
    out = dict(nseg=np.zeros(N, np.int32), tau=np.zeros(N), fails=np.zeros(N, np.int32))
    rc = _nblib.nbtrace_paths(_p(sites), sites.shape[0], _p(box), _p(rp), _p(cl), _p(rho), float(kappa),
                              _p(origins), _p(dirs), _p(st), N, int(threads), _p(out["nseg"]), _p(out["tau"]),
                              _p(out["fails"]))
    if rc:
        raise ValueError("nbtrace_paths: bad arguments")
    return out


def _bind(lib):
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_locate.argtypes = [P, I64, P, P, I64, P, P]
    lib.oracle_locate.restype = ctypes.c_int
    lib.oracle_trace.argtypes = [P, I64, P, P, ctypes.c_double, P, P, I64,
                                 ctypes.c_double, I64, P, P, P, P, P, P, P, P, P, P, ctypes.c_int, P]
    lib.oracle_trace.restype = ctypes.c_int
    lib.oracle_faces.argtypes = [P, I64, P, P, I64, I64, P, P, P, P, P]
    lib.oracle_faces.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_get_threads.restype = ctypes.c_int
    return lib


def load_library(path: str):
    """Load an oracle shared library built from (a variant of) oracle.c.
    The functions below take it as ``lib=``; the default is liboracle.so."""
    return _bind(ctypes.CDLL(path))


def _load(lib=None):
    global _lib
    if lib is not None:
        return lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def locate(sites, box, pts, lib=None):
    """Nearest site per point (lowest index on ties), -1 outside the box.
    Returns (cell int32[N], gap float64[N]) where gap is the distance from the
    point to the bisector plane of its two nearest sites."""
    sites = _f64(sites, (-1, 3))
    pts = _f64(pts, (-1, 3))
    box = _f64(box, (6,))
    N = pts.shape[0]
    cell = np.empty(N, np.int32)
    gap = np.empty(N, np.float64)
    rc = _load(lib).oracle_locate(_p(sites), sites.shape[0], _p(box), _p(pts), N, _p(cell), _p(gap))
    if rc:
        raise ValueError("oracle_locate: bad arguments")
    return cell, gap


def trace(sites, box, density, origins, dirs, kappa=1.0, cap=256, eta=ETA, segments=True,
          lib=None, enter=False):
    """Paths by brute force. Returns a dict of numpy arrays: nseg, tau, chord,
    status, n_near, min_gap, cell0, start_s and, if ``segments``, seg_cell /
    seg_len / seg_end (where each segment ends, measured from the origin) of
    shape (N, cap) (entries past nseg are undefined). ``enter``: rays from
    outside the box start where they enter it (start_s)."""
    sites = _f64(sites, (-1, 3))
    box = _f64(box, (6,))
    origins = _f64(origins, (-1, 3))
    dirs = _f64(dirs, (-1, 3))
    rho = None if density is None else _f64(density, (-1,))
    N = origins.shape[0]
    out = dict(
        nseg=np.zeros(N, np.int32), tau=np.zeros(N), chord=np.zeros(N),
        status=np.zeros(N, np.int32), n_near=np.zeros(N, np.int32),
        min_gap=np.zeros(N), cell0=np.zeros(N, np.int32), start_s=np.zeros(N))
    sc = sl = se = None
    if segments:
        sc = np.full((N, cap), -7, np.int32)
        sl = np.zeros((N, cap))
        se = np.zeros((N, cap))
    rc = _load(lib).oracle_trace(
        _p(sites), sites.shape[0], _p(box), _p(rho), float(kappa), _p(origins), _p(dirs), N,
        float(eta), int(cap), _p(sc), _p(sl), _p(se), _p(out["nseg"]), _p(out["tau"]), _p(out["chord"]),
        _p(out["status"]), _p(out["n_near"]), _p(out["min_gap"]), _p(out["cell0"]), 1 if enter else 0,
        _p(out["start_s"]))
    if rc:
        raise ValueError("oracle_trace: bad arguments")
    if segments:
        out["seg_cell"] = sc
        out["seg_len"] = sl
        out["seg_end"] = se
    return out


def faces(sites, box, cells, cap=128, lib=None, bboxes=False):
    """Faces of the listed cells: list of (nbr int32[], area float64[]) and
    volumes float64[]; with bboxes=True also the cells' bounding boxes
    (n x 6: xmin, ymin, zmin, xmax, ymax, zmax, from the face corners).
    Neighbour >= 0 is a site index, -1..-6 a wall."""
    sites = _f64(sites, (-1, 3))
    box = _f64(box, (6,))
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    n = cells.shape[0]
    nbr = np.zeros((n, cap), np.int32)
    area = np.zeros((n, cap))
    nface = np.zeros(n, np.int32)
    vol = np.zeros(n)
    bb = np.zeros((n, 6)) if bboxes else None
    rc = _load(lib).oracle_faces(_p(sites), sites.shape[0], _p(box), _p(cells), n, cap,
                              _p(nbr), _p(area), _p(nface), _p(vol), None if bb is None else _p(bb))
    if rc:
        raise ValueError("oracle_faces: bad arguments or out of memory")
    if np.any(nface > cap):
        raise ValueError("oracle_faces: face capacity exceeded")
    res = [(nbr[q, :nface[q]].copy(), area[q, :nface[q]].copy()) for q in range(n)]
    return (res, vol, bb) if bboxes else (res, vol)


def segments_of(out, ray):
    """(cells, lengths) of one ray from a ``trace`` result."""
    n = int(out["nseg"][ray])
    return out["seg_cell"][ray, :n].copy(), out["seg_len"][ray, :n].copy()
