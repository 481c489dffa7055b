"""Closed-form paths through tensor-product lattices.

TEST INFRASTRUCTURE ONLY.

For sites {x_i} x {y_j} x {z_k} the squared distance separates by axis, so
the nearest site is found independently on each axis and every Voronoi cell
is the cuboid between the midpoints of consecutive coordinates (the box
walls close the outermost cells). A straight path through such a grid is
the classic voxel walk of Amanatides & Woo (1987): on each axis the next
slab wall is (wall - r0_a) / k_a away, and the ray moves to the next slab
on the axis whose wall comes first. Nothing from the neighbour-list method
is used. Site index = (i * ny + j) * nz + k.
"""
from __future__ import annotations

import math
from bisect import bisect_left, bisect_right

import numpy as np


def _walls(c, lo, hi):
    c = [float(v) for v in c]
    return [lo] + [0.5 * (c[i] + c[i + 1]) for i in range(len(c) - 1)] + [hi]


def lattice_path(xs, ys, zs, box, r0, k):
    """(cells int list, lengths float list, L) for one ray; k is normalised
    here. A ray starting exactly on a cell wall starts in the slab it moves
    into; one running inside a wall (k_a = 0 there) takes the lower slab."""
    axes = [xs, ys, zs]
    n = [len(a) for a in axes]
    walls = [_walls(axes[a], float(box[a]), float(box[a + 3])) for a in range(3)]
    k = np.asarray(k, dtype=np.float64)
    k = k / math.sqrt(float(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]))
    r0 = [float(v) for v in r0]
    L = math.inf
    for a in range(3):
        if k[a] > 0:
            L = min(L, (box[a + 3] - r0[a]) / k[a])
        elif k[a] < 0:
            L = min(L, (box[a] - r0[a]) / k[a])
    idx = []
    for a in range(3):
        interior = walls[a][1:-1]
        if k[a] > 0:
            i = bisect_right(interior, r0[a])
        else:
            i = bisect_left(interior, r0[a])
        idx.append(min(max(i, 0), n[a] - 1))

    def nxt(a):
        if k[a] > 0:
            return (walls[a][idx[a] + 1] - r0[a]) / k[a] if idx[a] + 1 < n[a] else math.inf
        if k[a] < 0:
            return (walls[a][idx[a]] - r0[a]) / k[a] if idx[a] > 0 else math.inf
        return math.inf

    cells, lens = [], []
    s_c = 0.0
    t_next = [nxt(a) for a in range(3)]
    while L > 0:
        t = min(t_next)
        cell = (idx[0] * n[1] + idx[1]) * n[2] + idx[2]
        if t >= L:
            if L - s_c > 0:
                cells.append(cell)
                lens.append(L - s_c)
            break
        if t - s_c > 0:
            cells.append(cell)
            lens.append(t - s_c)
            s_c = t
        for a in range(3):
            if t_next[a] == t:
                idx[a] += 1 if k[a] > 0 else -1
                t_next[a] = nxt(a)
    return cells, lens, L
