"""The CPU baseline of the paper's own path loop (oracle/nbtrace.c, used
only to time that baseline) against the oracle (no GPU): with the exact
neighbour lists (faces of the clipped cells, walls included) it meets the
same number of cells on every ray free of near-ties, with the same optical
depth up to the rounding of its running point."""
import numpy as np

import oracle
from paper_1310_1854_amd import workloads as W


def _lists(w):
    faces, _ = oracle.faces(w.sites, w.box, np.arange(w.M))
    rp = np.zeros(w.M + 1, np.int64)
    col = []
    for i, (nbr, area) in enumerate(faces):
        col += [int(j) for j, a in zip(nbr, area) if a > 0]
        rp[i + 1] = len(col)
    return rp, np.array(col, np.int32)


def test_paper_loop_matches_the_oracle():
    w = W.uniform_cube(M=300, N=2000, seed=4401)
    rp, col = _lists(w)
    start, _ = oracle.locate(w.sites, w.box, w.origins)
    ref = oracle.trace(w.sites, w.box, w.density, w.origins, w.dirs, cap=64)
    for threads in (1, 4):
        got = oracle.nbtrace(w.sites, w.box, rp, col, w.density, w.origins, w.dirs, start, threads=threads)
        clean = ref["n_near"] == 0
        assert clean.sum() > 0.99 * w.N
        assert np.array_equal(got["nseg"][clean], ref["nseg"][clean])
        assert np.all(got["fails"] == 0)
        assert np.allclose(got["tau"][clean], ref["tau"][clean], rtol=1e-10, atol=0)


def test_paper_loop_on_a_lattice_has_the_closed_form_counts():
    from oracle.dda import lattice_path
    w = W.cubic_lattice(5, N=500, seed=4402)
    rp, col = _lists(w)
    start, _ = oracle.locate(w.sites, w.box, w.origins)
    got = oracle.nbtrace(w.sites, w.box, rp, col, np.ones(w.M), w.origins, w.dirs, start, threads=2)
    for r in range(w.N):
        c, l, L = lattice_path(w.meta["xs"], w.meta["ys"], w.meta["zs"], w.box, w.origins[r], w.dirs[r])
        assert got["nseg"][r] == len(c), r
        assert abs(got["tau"][r] - L) <= 1e-12 * L, r
