"""The GPU tests' path comparison (no GPU): for near-tie rays, where several
results are correct, the validity check accepts a correct path and rejects
a wrong cell, a wrong optical depth and a pair of cells that are not
neighbours. The oracle's own paths stand in for the GPU's."""
import json
import os

import numpy as np
import pytest

import oracle
from pathcmp import compare

HERE = os.path.dirname(os.path.abspath(__file__))


def _case():
    g = json.load(open(os.path.join(HERE, "golden", "hand_paths.json")))
    c = next(x for x in g["cases"] if x["name"] == "lattice_vertex_crossing")
    sites = np.array(c["sites"], float)
    box = np.array(c["box"], float)
    rho = np.array([1.0, 2.0, 3.0, 4.0])
    o = np.array([c["origin"]], float)
    d = np.array([c["dir"]], float)
    ref = oracle.trace(sites, box, rho, o, d, cap=8)
    assert ref["n_near"][0] >= 1                  # the ray passes the edge where four cells meet
    faces, _ = oracle.faces(sites, box, np.arange(4))
    rp = np.zeros(5, np.int64)
    col = []
    for i, (nbr, area) in enumerate(faces):
        mine = sorted(int(j) for j, a in zip(nbr, area) if a > 0)
        col += mine
        rp[i + 1] = len(col)
    geo = dict(sites=sites, box=box, density=rho, kappa=1.0, origins=o, dirs=d, nbr=(rp, np.array(col, np.int32)))
    n = int(ref["nseg"][0])
    p = dict(tau=ref["tau"].copy(), n_seg=ref["nseg"].copy(), status=ref["status"].astype(np.uint8),
             ray_off=np.array([0, n]), seg_cell=ref["seg_cell"][0, :n].copy(), seg_len=ref["seg_len"][0, :n].copy())
    return p, ref, geo


def test_correct_near_tie_path_passes():
    p, ref, geo = _case()
    st = compare(p, ref, 1e-12, geo=geo)
    assert st["near"] == 1 and st["near_segments"] == 2


def test_another_correct_path_passes():
    # through the shared edge the path may list a zero-length-adjacent cell for a sliver: cell 1 for 1e-12 of L
    p, ref, geo = _case()
    L = ref["chord"][0]
    cells, lens = list(p["seg_cell"]), list(p["seg_len"])
    sl = 1e-12 * L
    p["seg_cell"] = np.array([cells[0], 1, cells[1]])
    p["seg_len"] = np.array([lens[0] - sl, sl, lens[1]])
    p["n_seg"] = np.array([3])
    p["ray_off"] = np.array([0, 3])
    p["tau"] = np.array([1.0 * (lens[0] - sl) + 2.0 * sl + 4.0 * lens[1]])
    st = compare(p, ref, 1e-12, geo=geo)
    assert st["near_segments"] == 3


def test_wrong_cell_is_caught():
    p, ref, geo = _case()
    p["seg_cell"] = p["seg_cell"].copy()
    p["seg_cell"][1] = 1                           # a neighbour, but not the cell the second segment lies in
    p["tau"] = np.array([float(np.sum(geo["density"][p["seg_cell"]] * p["seg_len"]))])
    with pytest.raises(AssertionError):
        compare(p, ref, 1e-12, geo=geo)


def test_wrong_tau_is_caught():
    p, ref, geo = _case()
    p["tau"] = p["tau"] * (1.0 + 1e-9)
    with pytest.raises(AssertionError):
        compare(p, ref, 1e-12, geo=geo)


def test_cells_that_are_not_neighbours_are_caught():
    p, ref, geo = _case()
    # the path steps 0 -> 3 through the edge shared by all four cells (0 and 3 touch only there):
    # accepted through the neighbours 1 and 2 of both; with 3 unreachable from 0's neighbours it is not
    rp = np.array([0, 2, 3, 4, 4], np.int64)
    col = np.array([1, 2, 0, 0], np.int32)      # 0: {1, 2}; 1: {0}; 2: {0}; 3: {}
    geo["nbr"] = (rp, col)
    with pytest.raises(AssertionError):
        compare(p, ref, 1e-12, geo=geo)
