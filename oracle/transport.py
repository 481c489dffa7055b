"""Transport quantities along the oracle's paths (test infrastructure only).

Two plain definitions on top of a path (the ordered cells m_1..m_n with
lengths l_1..l_n and end positions s_1..s_n measured from the origin, as
``oracle.trace`` returns them):

* Interaction point (the paths serve the photon-package transport of the
  test simulations, Sect. 3.4, where packages scatter and dust absorption
  and the radiation field are tallied on the grid; the paper does not spell
  the sampling out, so the standard Monte Carlo step is used: a package
  travels until the optical depth drawn for it, -ln u, is used up):
  with tau_k = tau_{k-1} + (kappa rho_{m_k}) l_k (tau_0 = 0, the order in
  which tau is summed everywhere), the package interacts in the first cell
  m_k with kappa rho_{m_k} > 0 and tau_k >= tau_stop, at the distance
  s_{k-1} + (tau_stop - tau_{k-1}) / (kappa rho_{m_k}) from the origin
  (s_0 = 0); the path is cut there, its last segment shortened to that
  point. A non-positive tau_stop interacts where the path starts (the
  origin, or where a ray from outside enters the box), in the start cell,
  before any segment; a package that reaches the wall first escapes (cell
  -1, distance L).

* Per-cell tallies of the path up to where it ends (the interaction point
  or the wall), with a weight w per ray: the path length w l_k deposited in
  cell m_k, and the luminosity absorbed there under continuous absorption,
  w exp(-tau_{k-1}) (1 - exp(-kappa rho_{m_k} l_k)) -- the fraction of the
  package that is absorbed inside the cell. Summed over a path the second
  telescopes to w (1 - exp(-tau_n)).

Everything here is pure Python over the oracle's segments: obviously
correct, slow, for small inputs.
"""
from __future__ import annotations

import math

import numpy as np


def interaction(cells, lens, ends, rho, kappa, tau_stop, cell0, chord, s0=0.0):
    """Interaction point of one path starting at distance s0 from the origin
    (0 unless it entered the box from outside): (cell, distance, number of
    segments kept, tau at the end, length of the last kept segment)."""
    if tau_stop <= 0.0:
        return int(cell0), s0, 0, 0.0, None
    tau = 0.0
    s_prev = s0
    for k in range(len(cells)):
        m = int(cells[k])
        kr = kappa * rho[m]
        tn = tau + kr * lens[k]
        if kr > 0.0 and tn >= tau_stop:
            lp = (tau_stop - tau) / kr
            return m, s_prev + lp, k + 1, tau + kr * lp, lp
        tau = tn
        s_prev = ends[k]
    return -1, float(chord), len(cells), tau, None


def interactions(res, rho, kappa, tau_stop):
    """Interaction points of every ray of an ``oracle.trace`` result (with
    segments): dict of numpy arrays cell, s, nseg, tau, and the shortened
    last length (NaN where the path is not cut)."""
    N = res["nseg"].shape[0]
    out = dict(cell=np.zeros(N, np.int32), s=np.zeros(N), nseg=np.zeros(N, np.int32), tau=np.zeros(N),
               last_len=np.full(N, np.nan))
    rho = np.asarray(rho, dtype=np.float64)
    for i in range(N):
        if res["status"][i] != 0:
            out["cell"][i] = -1
            continue
        n = int(res["nseg"][i])
        c, s, k, t, lp = interaction(res["seg_cell"][i, :n], res["seg_len"][i, :n], res["seg_end"][i, :n], rho,
                                     kappa, float(tau_stop[i]), res["cell0"][i], res["chord"][i],
                                     float(res["start_s"][i]))
        out["cell"][i], out["s"][i], out["nseg"][i], out["tau"][i] = c, s, k, t
        if lp is not None:
            out["last_len"][i] = lp
    return out


def tallies(res, rho, kappa, M, weight=None, tau_stop=None):
    """Per-cell path-length and absorbed-luminosity tallies (user order) of
    the paths of an ``oracle.trace`` result, cut at the interaction points
    when tau_stop is given."""
    rho = np.asarray(rho, dtype=np.float64)
    t_len = np.zeros(M)
    t_abs = np.zeros(M)
    N = res["nseg"].shape[0]
    for i in range(N):
        if res["status"][i] != 0:
            continue
        w = 1.0 if weight is None else float(weight[i])
        n = int(res["nseg"][i])
        cells, lens = res["seg_cell"][i, :n], res["seg_len"][i, :n]
        if tau_stop is not None:
            c, s, k, t, lp = interaction(cells, lens, res["seg_end"][i, :n], rho, kappa, float(tau_stop[i]),
                                         res["cell0"][i], res["chord"][i], float(res["start_s"][i]))
            n = k
            lens = np.array(lens[:n], dtype=np.float64)
            if lp is not None:
                lens[n - 1] = lp
        tau = 0.0
        for k in range(n):
            m = int(cells[k])
            dt = kappa * rho[m] * lens[k]
            t_len[m] += w * lens[k]
            t_abs[m] += w * math.exp(-tau) * -math.expm1(-dt)
            tau = tau + dt
    return t_len, t_abs
