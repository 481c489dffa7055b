"""Pins of the oracle's transport quantities (oracle/transport.py):
interaction points and per-cell tallies along the oracle's paths, checked
against closed forms, a telescoping identity and the voxel walk of a
lattice, plus planted mistakes that each pin catches."""
import importlib.util
import math
import os

import numpy as np
import pytest

import oracle
from oracle import transport as T
from oracle.dda import lattice_path
from paper_1310_1854_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _slab(rho):
    """The three-collinear-sites case of tests/golden/hand_paths.json: cells
    split at x = 1 and 2.5; the ray from (0.25, 0.5, 0.25) along (4, 0, 3)/5
    crosses x = 1 at s = 0.9375 and leaves through z = 1 at L = 1.25, so the
    path is (0, 0.9375), (1, 0.3125)."""
    sites = np.array([[0.5, 0.5, 0.5], [1.5, 0.5, 0.5], [3.5, 0.5, 0.5]])
    box = [0, 0, 0, 4, 1, 1]
    res = oracle.trace(sites, box, np.array(rho, float), [[0.25, 0.5, 0.25]], [[4.0, 0.0, 3.0]], cap=8)
    assert list(res["seg_cell"][0, :2]) == [0, 1] and res["seg_end"][0, 0] == 0.9375
    return res


def test_interaction_single_cell_closed_form():
    # one site: the cell is the box; kappa rho = 1, so the interaction lies at s = tau_stop
    res = oracle.trace([[0.5, 0.5, 0.5]], [0, 0, 0, 1, 1, 1], [2.0], [[0.1, 0.2, 0.3]] * 4, [[1, 0, 0]] * 4,
                       kappa=0.5, cap=4)
    out = T.interactions(res, [2.0], 0.5, np.array([0.4, 2.0, 0.0, -1.0]))
    assert list(out["cell"]) == [0, -1, 0, 0]
    assert list(out["s"]) == [0.4, 0.9, 0.0, 0.0]
    assert list(out["nseg"]) == [1, 1, 0, 0]
    assert out["last_len"][0] == 0.4 and np.isnan(out["last_len"][1])


def test_interaction_slab_closed_form():
    res = _slab([2, 3, 5])
    # tau after the segments: 2 * 0.9375 = 1.875, then 1.875 + 3 * 0.3125 = 2.8125
    ts = np.array([1.0, 1.875, 2.0, 3.0])
    out = T.interactions({k: np.repeat(v, 4, axis=0) for k, v in res.items()}, [2, 3, 5], 1.0, ts)
    assert list(out["cell"]) == [0, 0, 1, -1]
    assert out["s"][0] == 0.5                       # 1.0 / 2
    assert out["s"][1] == 0.9375                    # used up exactly at the first boundary: still cell 0
    assert abs(out["s"][2] - (0.9375 + 0.125 / 3.0)) < 1e-15
    assert out["s"][3] == 1.25                      # escapes through the wall at L
    assert list(out["nseg"]) == [1, 1, 2, 2]
    assert out["tau"][3] == 2.8125


def test_interaction_skips_empty_cells():
    res = _slab([2, 0, 5])
    out = T.interactions(res, [2, 0, 5], 1.0, np.array([1.9]))
    assert out["cell"][0] == -1 and out["s"][0] == 1.25     # the middle cell has no dust


def _cube(seed, M=150, N=250):
    w = W.uniform_cube(M=M, N=N, seed=seed)
    res = oracle.trace(w.sites, w.box, w.density, w.origins, w.dirs, cap=64)
    return w, res


def test_tally_totals_telescope():
    w, res = _cube(5)
    wt = np.random.default_rng(3).uniform(0.5, 2.0, w.N)
    t_len, t_abs = T.tallies(res, w.density, 1.3, w.M, weight=wt)
    res13 = oracle.trace(w.sites, w.box, w.density, w.origins, w.dirs, kappa=1.3, cap=64)
    ok = res13["status"] == 0
    assert abs(t_len.sum() - (wt * res13["chord"])[ok].sum()) <= 1e-12 * t_len.sum()
    # absorbed fractions along a path telescope to 1 - exp(-tau)
    want = (wt * -np.expm1(-res13["tau"]))[ok].sum()
    assert abs(t_abs.sum() - want) <= 1e-12 * want


def test_tally_totals_with_interactions():
    w, res = _cube(6)
    ts = -np.log(np.random.default_rng(4).uniform(size=w.N))
    out = T.interactions(res, w.density, 1.0, ts)
    t_len, t_abs = T.tallies(res, w.density, 1.0, w.M, tau_stop=ts)
    ok = res["status"] == 0
    stopped = ok & (out["cell"] >= 0)
    assert stopped.sum() > 0 and (ok & (out["cell"] < 0)).sum() > 0
    # a cut path deposits exactly 1 - exp(-tau_stop); an escaping one 1 - exp(-tau)
    want = (-np.expm1(-np.where(stopped, ts, res["tau"])))[ok].sum()
    assert abs(t_abs.sum() - want) <= 1e-12 * want
    assert abs(t_len.sum() - out["s"][ok].sum()) <= 1e-12 * t_len.sum()


def test_tally_lattice_matches_voxel_walk():
    w = W.random_tensor_lattice((5, 4, 6), N=200)
    res = oracle.trace(w.sites, w.box, w.density, w.origins, w.dirs, cap=64)
    t_len, _ = T.tallies(res, w.density, 1.0, w.M)
    ref = np.zeros(w.M)
    for r in range(w.N):
        cells, lens, _ = lattice_path(w.meta["xs"], w.meta["ys"], w.meta["zs"], w.box, w.origins[r], w.dirs[r])
        for c, l in zip(cells, lens):
            ref[c] += l
    assert np.max(np.abs(t_len - ref)) <= 1e-12 * max(ref.max(), 1.0)


# planted mistakes: each must fail at least one pin above
MUTANTS = {
    "tau_order": ("tn = tau + kr * lens[k]", "tn = tau + kr * lens[k] * 1.0000001"),
    "no_prev_end": ("        s_prev = ends[k]", "        s_prev = s_prev"),
    "strict_stop": ("tn >= tau_stop", "tn > tau_stop"),
    "wrong_cut": ("lp = (tau_stop - tau) / kr", "lp = tau_stop / kr"),
    "abs_after": ("w * math.exp(-tau) * -math.expm1(-dt)", "w * math.exp(-tau - dt) * -math.expm1(-dt)"),
    "stop_start": ("if tau_stop <= 0.0:", "if tau_stop < 0.0:"),
    "tally_uncut": ("                lens[n - 1] = lp", "                pass"),
}


def _mutant(name):
    src = open(T.__file__).read()
    a, b = MUTANTS[name]
    assert a in src, name
    spec = importlib.util.spec_from_loader(f"transport_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src.replace(a, b), f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


PINS = [test_interaction_single_cell_closed_form, test_interaction_slab_closed_form,
        test_interaction_skips_empty_cells, test_tally_totals_telescope, test_tally_totals_with_interactions,
        test_tally_lattice_matches_voxel_walk]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    mod = _mutant(name)
    caught = False
    for pin in PINS:
        monkeypatch.setattr(T, "interaction", mod.interaction)
        monkeypatch.setattr(T, "interactions", mod.interactions)
        monkeypatch.setattr(T, "tallies", mod.tallies)
        try:
            pin()
        except AssertionError:
            caught = True
            break
        finally:
            monkeypatch.undo()
    assert caught, f"mutant {name} passes every pin"
