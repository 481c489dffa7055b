"""Exact rational paths by a sweep over all pairwise bisector crossings.

TEST INFRASTRUCTURE ONLY. Tiny inputs (tens of sites): cost O(M^3) in
Python fractions.

This is an independent route to the same definition as ``oracle.c``: along
the line r(t) = r0 + t k the squared distance to site j is
    |r0 - p_j|^2 + 2 t k.(r0 - p_j) + t^2 |k|^2,
whose quadratic term is common to all sites, so the nearest site can only
change at a root of the difference of two of these linear functions (a
bisector crossing, Sect. 2.2, Eqs. 1-4). All such roots in (0, T) are
collected, the nearest site is evaluated exactly at the midpoint of every
interval between consecutive roots (Sect. 2.1's definition of a cell), and
runs with the same site are merged. No step of the neighbour-list method is
used. FP64 inputs are dyadic rationals, so every value here is exact; the
direction k is not normalised (its length is irrational in general) and
lengths are returned in units of t, i.e. multiplied by |k| to get distance.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from typing import List, Sequence, Tuple


def exact_chord(box, r0, k) -> Fr:
    """Parameter T at which r0 + t k leaves the box (Eq. 5 on every axis)."""
    T = None
    for a in range(3):
        if k[a] > 0:
            s = (box[a + 3] - r0[a]) / k[a]
        elif k[a] < 0:
            s = (box[a] - r0[a]) / k[a]
        else:
            continue
        if T is None or s < T:
            T = s
    return T


def exact_path(sites: Sequence[Sequence[float]], box: Sequence[float],
               r0: Sequence[float], k: Sequence[float]) -> Tuple[List[Tuple[int, Fr]], Fr]:
    """Ordered list of (cell, length in units of t) and the exit parameter T.
    Inside an interval on which two sites stay equally near for its whole
    length (the ray lies in their bisector plane) the lower index is taken."""
    P = [[Fr(x) for x in p] for p in sites]
    R = [Fr(x) for x in r0]
    K = [Fr(x) for x in k]
    B = [Fr(x) for x in box]
    for a in range(3):
        if not (B[a] <= R[a] <= B[a + 3]):
            raise ValueError("origin outside the box")
    T = exact_chord(B, R, K)
    if T is None:
        raise ValueError("zero direction")
    M = len(P)
    a_ = [sum((R[c] - p[c]) ** 2 for c in range(3)) for p in P]
    b_ = [2 * sum(K[c] * (R[c] - p[c]) for c in range(3)) for p in P]
    cuts = {Fr(0), T}
    for i in range(M):
        for j in range(i + 1, M):
            db = b_[i] - b_[j]
            if db != 0:
                t = (a_[j] - a_[i]) / db
                if 0 < t < T:
                    cuts.add(t)
    cuts = sorted(cuts)
    path: List[Tuple[int, Fr]] = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        mid = (lo + hi) / 2
        best, bv = -1, None
        for j in range(M):
            v = a_[j] + b_[j] * mid
            if bv is None or v < bv:
                best, bv = j, v
        if path and path[-1][0] == best:
            path[-1] = (best, path[-1][1] + (hi - lo))
        else:
            path.append((best, hi - lo))
    return path, T


def exact_tau(path, rho, kappa=1.0) -> Fr:
    """kappa * sum(rho_m * length_m) in units of t, exactly."""
    return Fr(kappa) * sum(Fr(float(rho[m])) * dt for m, dt in path)
