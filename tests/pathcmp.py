"""Comparison of GPU paths with oracle paths (used by the GPU tests).

Bar: on rays the oracle finds free of near-ties (no two candidate crossings
within 1e-9 of the chord at any step, and a start point at least that far
from a cell boundary) the cell sequences must be identical and every
segment length and the optical depth must agree to the stated relative
tolerance (lengths relative to the chord L, tau relative to itself). Rays
with near-ties may legitimately list a different cell for a sliver (several
results are correct); for them the status and the total length are
compared and, given the geometry (``geo``), the path is checked for being
one of the correct ones: each segment's midpoint is no farther from its
listed cell's site than from the nearest site (Sect. 2.1: a cell holds the
points nearest its site) by more than the near-tie allowance, consecutive
cells are neighbours in the grid's lists (or neighbours of a neighbour,
where the path passes an edge or vertex), tau is kappa times the sum of
rho times length over the listed segments, and it differs from the
oracle's by no more than the slivers can account for.
"""
from __future__ import annotations

import numpy as np


def gpu_paths(out: dict) -> dict:
    """Copy a vrt.trace result to numpy."""
    res = {k: out[k].cpu().numpy() for k in ("tau", "n_seg", "status", "n_fallback")}
    if "seg_cell" in out:
        res["ray_off"] = out["ray_off"].cpu().numpy()
        res["seg_cell"] = out["seg_cell"].cpu().numpy()
        res["seg_len"] = out["seg_len"].cpu().numpy()
    return res


def ray_segments(p: dict, r: int):
    n = int(p["n_seg"][r])
    o = int(p["ray_off"][r])
    return p["seg_cell"][o:o + n], p["seg_len"][o:o + n]


ETA = 1e-9   # the oracle's near-tie threshold, relative to the chord


def check_near_tie_paths(p: dict, ref: dict, geo: dict, pairs, tol: float) -> int:
    """The validity bar for near-tie rays (see the module docstring). geo:
    sites, box, density, kappa, origins and dirs of the oracle's rays, and
    nbr = (row_ptr, col), the grid's neighbour lists in user order (walls
    negative). pairs: (oracle ray i, GPU ray r). Returns the segments
    checked."""
    import oracle
    sites = np.asarray(geo["sites"], np.float64)
    rho = np.asarray(geo["density"], np.float64)
    kappa = float(geo.get("kappa", 1.0))
    rp, col = geo["nbr"]
    mids, owner, listed, allow = [], [], [], []
    for i, r in pairs:
        cells, lens = ray_segments(p, r)
        if len(cells) == 0:
            continue
        L = ref["chord"][i]
        k = np.asarray(geo["dirs"][i], np.float64)
        k = k / np.linalg.norm(k)
        s = ref["start_s"][i] + np.concatenate([[0.0], np.cumsum(lens)[:-1]]) + 0.5 * lens
        mids.append(np.asarray(geo["origins"][i], np.float64)[None, :] + s[:, None] * k[None, :])
        owner.append(np.full(len(cells), i))
        listed.append(np.asarray(cells, np.int64))
        allow.append(np.full(len(cells), 4.0 * ETA * L + 1e-12 * L))
        # consecutive cells are neighbours in the grid's lists, or neighbours of one neighbour: a path
        # through an edge or vertex where cells meet passes the cells between them with zero length
        for a, b in zip(cells[:-1], cells[1:]):
            na = col[rp[a]:rp[a + 1]]
            ok = b in na or any(b in col[rp[c]:rp[c + 1]] for c in na if c >= 0)
            assert ok, f"ray {r}: cells {a} and {b} are not neighbours"
        # tau is kappa rho l summed over the listed segments, and close to the oracle's
        t = float(p["tau"][r])
        t_own = kappa * float(np.sum(rho[cells] * lens))
        assert abs(t - t_own) <= max(tol, 1e-12) * max(abs(t_own), 1e-300) * 4, f"ray {r}: tau {t} vs {t_own}"
        sliver = 4.0 * ETA * L * kappa * float(rho.max()) * max(int(ref["n_near"][i]), 1)
        assert abs(t - ref["tau"][i]) <= tol * abs(ref["tau"][i]) + sliver, f"ray {r}: tau vs the oracle's"
    if not mids:
        return 0
    x = np.concatenate(mids)
    c = np.concatenate(listed)
    near, _ = oracle.locate(sites, geo["box"], x)
    d_listed = np.linalg.norm(x - sites[c], axis=1)
    d_near = np.linalg.norm(x - sites[near], axis=1)
    bad = d_listed - d_near > np.concatenate(allow)
    assert not bad.any(), f"{int(bad.sum())} segment midpoints are not in their listed cell"
    return int(x.shape[0])


def compare(p: dict, ref: dict, tol: float, idx=None, geo=None) -> dict:
    """Assert the parity bar for oracle ray i against GPU ray idx[i]
    (idx = identity by default); return statistics. With ``geo`` (see
    check_near_tie_paths) near-tie rays are checked for validity as well."""
    N = ref["nseg"].shape[0]
    idx = np.arange(N) if idx is None else np.asarray(idx)
    have_segs = "seg_cell" in p
    max_dl = max_dtau = 0.0
    n_clean = n_near = 0
    near_pairs = []
    for i in range(N):
        r = int(idx[i])
        assert int(p["status"][r]) == int(ref["status"][i]), f"ray {r}: status {p['status'][r]} vs {ref['status'][i]}"
        if ref["status"][i] != 0:
            continue
        L = ref["chord"][i]
        if ref["n_near"][i] > 0:
            n_near += 1
            if have_segs:
                _, lens = ray_segments(p, r)
                assert abs(lens.sum() - (L - ref["start_s"][i])) <= 4 * max(tol, 1e-12) * max(L, 1e-300), \
                    f"ray {r}: total length"
                near_pairs.append((i, r))
            continue
        n_clean += 1
        assert p["n_seg"][r] == ref["nseg"][i], f"ray {r}: {p['n_seg'][r]} vs {ref['nseg'][i]} segments"
        t0, t1 = float(p["tau"][r]), float(ref["tau"][i])
        dt = abs(t0 - t1) / max(abs(t1), 1e-300)
        assert dt <= tol, f"ray {r}: tau {t0} vs {t1}"
        max_dtau = max(max_dtau, dt)
        if have_segs:
            cells, lens = ray_segments(p, r)
            n = int(p["n_seg"][r])
            assert np.array_equal(cells, ref["seg_cell"][i, :n]), f"ray {r}: cell sequence differs"
            if n:
                dl = float(np.max(np.abs(lens - ref["seg_len"][i, :n]))) / max(L, 1e-300)
                assert dl <= tol, f"ray {r}: segment length differs by {dl} L"
                max_dl = max(max_dl, dl)
    checked = check_near_tie_paths(p, ref, geo, near_pairs, tol) if (geo is not None and near_pairs) else 0
    return dict(max_len_diff=max_dl, max_tau_diff=max_dtau, clean=n_clean, near=n_near, near_segments=checked)
