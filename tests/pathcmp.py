"""Comparison of GPU paths with oracle paths (used by the GPU tests).

Bar: on rays the oracle finds free of near-ties (no two candidate crossings
within 1e-9 of the chord at any step, and a start point at least that far
from a cell boundary) the cell sequences must be identical and every
segment length and the optical depth must agree to the stated relative
tolerance (lengths relative to the chord L, tau relative to itself). Rays
with near-ties may legitimately list a different cell for a sliver; for them
only the total length and the status are compared.
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


def compare(p: dict, ref: dict, tol: float, idx=None) -> dict:
    """Assert the parity bar for oracle ray i against GPU ray idx[i]
    (idx = identity by default); return statistics."""
    N = ref["nseg"].shape[0]
    idx = np.arange(N) if idx is None else np.asarray(idx)
    have_segs = "seg_cell" in p
    max_dl = max_dtau = 0.0
    n_clean = n_near = 0
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
                assert abs(lens.sum() - L) <= 4 * max(tol, 1e-12) * max(L, 1e-300), f"ray {r}: total length"
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
    return dict(max_len_diff=max_dl, max_tau_diff=max_dtau, clean=n_clean, near=n_near)
