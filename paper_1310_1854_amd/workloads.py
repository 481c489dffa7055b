"""Seeded synthetic inputs: site sets, per-cell densities and rays.

This module only draws random numbers and evaluates the synthetic density
fields; it holds none of the path computation. Both the product path and the
test oracle consume what it returns, so neither depends on the other.

The site sets stand in for the paper's model shapes (Sect. 3.2: a uniform
site cloud, density-weighted sites in a disc, a 1/r-weighted disc as in the
Pascucci set-up of Sect. 3.5); none of the paper's own model data is used.

Every generator takes an integer ``seed`` and derives four independent
streams from ``numpy.random.SeedSequence(seed).spawn(4)``:
``[sites, density, origins, directions]``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 20131854


@dataclasses.dataclass
class Workload:
    """A grid (box + sites + per-cell density) and a batch of rays."""

    name: str
    box: np.ndarray          # (6,) float64: xmin, ymin, zmin, xmax, ymax, zmax
    sites: np.ndarray        # (M, 3) float64, C-contiguous
    density: np.ndarray      # (M,) float64
    origins: np.ndarray      # (N, 3) float64
    dirs: np.ndarray         # (N, 3) float64, unit length
    kappa: float = 1.0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.sites.shape[0])

    @property
    def N(self) -> int:
        return int(self.origins.shape[0])

    def subsample(self, n: int, seed: int = 7, split: int = None) -> "Workload":
        """Same grid, a seeded subset of ``n`` rays (for CPU-side checks).
        With ``split``, n // 2 rays from [0, split) and the rest from
        [split, N) (e.g. the flared disc's central and site-origin rays)."""
        n = min(int(n), self.N)
        rng = np.random.default_rng(seed)
        if split is None:
            idx = np.sort(rng.choice(self.N, size=n, replace=False))
        else:
            a = rng.choice(split, size=min(n // 2, split), replace=False)
            b = split + rng.choice(self.N - split, size=min(n - a.size, self.N - split), replace=False)
            idx = np.sort(np.concatenate([a, b]))
        return dataclasses.replace(
            self, origins=np.ascontiguousarray(self.origins[idx]),
            dirs=np.ascontiguousarray(self.dirs[idx]),
            meta=dict(self.meta, ray_index=idx))


def _streams(seed: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]


def isotropic_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere: z = 2u - 1, phi = 2 pi v."""
    z = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * math.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    d = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.ascontiguousarray(d)


def uniform_in_box(rng: np.random.Generator, n: int, box) -> np.ndarray:
    lo = np.asarray(box[:3], dtype=np.float64)
    hi = np.asarray(box[3:], dtype=np.float64)
    return np.ascontiguousarray(lo + rng.random((n, 3)) * (hi - lo))


def _dedupe_check(sites: np.ndarray) -> None:
    u = np.unique(sites, axis=0)
    if u.shape[0] != sites.shape[0]:
        raise RuntimeError("generator produced duplicate sites")


# --------------------------------------------------------------------------
# Configuration 0: uniform cube (the FP64 correctness case)
# --------------------------------------------------------------------------

def uniform_cube(M: int = 1000, N: int = 10_000, seed: int = SEED_BASE + 0,
                 half: float = 1.0) -> Workload:
    """M i.i.d. uniform sites in [-half, half]^3, density U[0,1], N rays with
    uniform origins in the box and isotropic directions, kappa = 1."""
    rs, rd, ro, rk = _streams(seed)
    box = np.array([-half] * 3 + [half] * 3, dtype=np.float64)
    sites = uniform_in_box(rs, M, box)
    density = rd.random(M)
    origins = uniform_in_box(ro, N, box)
    dirs = isotropic_dirs(rk, N)
    return Workload("uniform_cube", box, sites, density, origins, dirs, 1.0,
                    dict(seed=seed, M=M, N=N))


# --------------------------------------------------------------------------
# Configuration 1: exponential disc, rays from random sites
# --------------------------------------------------------------------------

def exp_disc_density(p: np.ndarray, hR: float = 2.5, hz: float = 0.3) -> np.ndarray:
    R = np.hypot(p[:, 0], p[:, 1])
    return np.exp(-R / hR - np.abs(p[:, 2]) / hz)


def exp_disc(M: int = 100_000, N: int = 1_000_000, seed: int = SEED_BASE + 1,
             hR: float = 2.5, hz: float = 0.3) -> Workload:
    """Sites drawn with probability proportional to exp(-R/hR - |z|/hz) in
    [-10,10]^2 x [-3,3]; cell density evaluated at the site (unnormalised);
    rays start at sites chosen uniformly with replacement, isotropic."""
    rs, rd, ro, rk = _streams(seed)
    box = np.array([-10.0, -10.0, -3.0, 10.0, 10.0, 3.0])
    out = np.empty((0, 3))
    while out.shape[0] < M:
        n = int((M - out.shape[0]) * 1.2) + 64
        R = rs.gamma(2.0, hR, n)          # pdf(R) ~ R exp(-R/hR)
        phi = 2.0 * math.pi * rs.random(n)
        z = rs.laplace(0.0, hz, n)
        p = np.stack([R * np.cos(phi), R * np.sin(phi), z], axis=1)
        ok = (np.abs(p[:, 0]) <= 10.0) & (np.abs(p[:, 1]) <= 10.0) & (np.abs(p[:, 2]) <= 3.0)
        out = np.concatenate([out, p[ok]])
    sites = np.ascontiguousarray(out[:M])
    density = exp_disc_density(sites, hR, hz)
    origins = np.ascontiguousarray(sites[ro.integers(0, M, N)])
    dirs = isotropic_dirs(rk, N)
    return Workload("exp_disc", box, sites, density, origins, dirs, 1.0,
                    dict(seed=seed, M=M, N=N, hR=hR, hz=hz))


# --------------------------------------------------------------------------
# Configuration 2: flared 1/R disc (Pascucci-like shape), point source + sites
# --------------------------------------------------------------------------

def flared_disc_density(p: np.ndarray, R0: float = 500.0, Rin: float = 1.0,
                        Rout: float = 1000.0) -> np.ndarray:
    R = np.hypot(p[:, 0], p[:, 1])
    Rs = np.maximum(R, 1e-300)
    h = 0.125 * R0 * (Rs / R0) ** 1.125
    rho = (Rs / R0) ** -1.0 * np.exp(-(math.pi / 4.0) * (p[:, 2] / h) ** 2)
    return np.where((R >= Rin) & (R <= Rout), rho, 0.0)


def flared_disc(M: int = 1_000_000, N: int = 8_000_000, seed: int = SEED_BASE + 2,
                R0: float = 500.0, uniform_frac: float = 0.01) -> Workload:
    """99% of sites from rho ~ (R/R0)^-1 exp(-(pi/4)(z/h)^2), h = 0.125 R0 (R/R0)^1.125,
    R in [1, 1000] AU; 1% uniform in the box +-1000 AU. R0 = 500 AU is a free
    choice (the shape formula leaves it open). Half of the rays start at the
    centre (0,0,0), half at sites chosen uniformly; isotropic directions."""
    rs, rd, ro, rk = _streams(seed)
    box = np.array([-1000.0] * 3 + [1000.0] * 3)
    n_uni = int(round(M * uniform_frac))
    n_disc = M - n_uni
    a = 2.125                                    # pdf(R) ~ R^1.125 -> CDF ~ R^2.125
    out = np.empty((0, 3))
    while out.shape[0] < n_disc:
        n = int((n_disc - out.shape[0]) * 1.05) + 64
        u = rs.random(n)
        R = (1.0 + u * (1000.0 ** a - 1.0)) ** (1.0 / a)
        h = 0.125 * R0 * (R / R0) ** 1.125
        z = rs.normal(0.0, 1.0, n) * h * math.sqrt(2.0 / math.pi)
        phi = 2.0 * math.pi * rs.random(n)
        p = np.stack([R * np.cos(phi), R * np.sin(phi), z], axis=1)
        ok = np.all(np.abs(p) <= 1000.0, axis=1)
        out = np.concatenate([out, p[ok]])
    disc = out[:n_disc]
    uni = uniform_in_box(rs, n_uni, box)
    sites = np.ascontiguousarray(np.concatenate([disc, uni]))
    density = flared_disc_density(sites, R0)
    n_c = N // 2
    origins = np.concatenate([np.zeros((n_c, 3)), sites[ro.integers(0, M, N - n_c)]])
    dirs = isotropic_dirs(rk, N)
    return Workload("flared_disc", box, sites, density, np.ascontiguousarray(origins), dirs, 1.0,
                    dict(seed=seed, M=M, N=N, R0=R0, n_central=n_c))


# --------------------------------------------------------------------------
# Configuration 3: clumpy medium, rays from clumps and from the box faces
# --------------------------------------------------------------------------

def clumpy(M: int = 4_000_000, N: int = 10_000_000, seed: int = SEED_BASE + 3,
           n_clumps: int = 2000, clump_frac: float = 0.5, bg_scale: float = 0.5) -> Workload:
    """Box [-1,1]^3. Half the sites in 2000 Gaussian clumps (sigma log-uniform in
    [0.01, 0.05] x box side, masses log-uniform in [1, 100], sites per clump
    proportional to mass, centres inset by 2 sigma); half from a smooth
    background ~ exp(-|x|/0.5). Cell density = background + the 8 nearest
    clumps' Gaussians at the site. Half of the rays start inside clumps (clump
    chosen by mass, offset ~ N(0, sigma)), half uniformly on the box faces
    with isotropic inward directions."""
    from scipy.spatial import cKDTree

    rs, rd, ro, rk = _streams(seed)
    box = np.array([-1.0] * 3 + [1.0] * 3)
    side = 2.0
    sig = side * np.exp(rd.uniform(math.log(0.01), math.log(0.05), n_clumps))
    mass = np.exp(rd.uniform(math.log(1.0), math.log(100.0), n_clumps))
    cen = -1.0 + 2.0 * sig[:, None] + rd.random((n_clumps, 3)) * (2.0 - 4.0 * sig[:, None])
    n_clump_sites = int(round(M * clump_frac))
    counts = rs.multinomial(n_clump_sites, mass / mass.sum())
    pts = []
    owner = np.repeat(np.arange(n_clumps), counts)
    p = cen[owner] + rs.normal(0.0, 1.0, (n_clump_sites, 3)) * sig[owner][:, None]
    bad = ~np.all(np.abs(p) <= 1.0, axis=1)
    while bad.any():
        nb = int(bad.sum())
        p[bad] = cen[owner[bad]] + rs.normal(0.0, 1.0, (nb, 3)) * sig[owner[bad]][:, None]
        bad = ~np.all(np.abs(p) <= 1.0, axis=1)
    pts.append(p)
    n_bg = M - n_clump_sites
    got = np.empty((0, 3))
    while got.shape[0] < n_bg:
        n = int((n_bg - got.shape[0]) * 1.3) + 64
        r = rs.gamma(3.0, bg_scale, n)             # pdf(r) ~ r^2 exp(-r/scale)
        d = isotropic_dirs(rs, n)
        q = d * r[:, None]
        got = np.concatenate([got, q[np.all(np.abs(q) <= 1.0, axis=1)]])
    pts.append(got[:n_bg])
    sites = np.ascontiguousarray(np.concatenate(pts))

    def field(x):
        bg = np.exp(-np.linalg.norm(x, axis=1) / bg_scale)
        tree = cKDTree(cen)
        k = min(8, n_clumps)
        _, idx = tree.query(x, k=k)
        idx = idx.reshape(x.shape[0], k)
        s = sig[idx]
        d2 = np.sum((x[:, None, :] - cen[idx]) ** 2, axis=2)
        amp = mass[idx] / (n_clumps * (2.0 * math.pi * s * s) ** 1.5)
        return bg + np.sum(amp * np.exp(-0.5 * d2 / (s * s)), axis=1)

    density = np.empty(M)
    step = 1 << 20
    for i in range(0, M, step):
        density[i:i + step] = field(sites[i:i + step])

    n_in = N // 2
    cl = ro.choice(n_clumps, size=n_in, p=mass / mass.sum())
    o_in = cen[cl] + ro.normal(0.0, 1.0, (n_in, 3)) * sig[cl][:, None]
    bad = ~np.all(np.abs(o_in) <= 1.0, axis=1)
    while bad.any():
        nb = int(bad.sum())
        o_in[bad] = cen[cl[bad]] + ro.normal(0.0, 1.0, (nb, 3)) * sig[cl[bad]][:, None]
        bad = ~np.all(np.abs(o_in) <= 1.0, axis=1)
    n_face = N - n_in
    face = ro.integers(0, 6, n_face)
    o_f = -1.0 + 2.0 * ro.random((n_face, 3))
    ax = face // 2
    sgn = np.where(face % 2 == 0, -1.0, 1.0)
    o_f[np.arange(n_face), ax] = sgn
    d_in = isotropic_dirs(rk, n_in)
    d_f = isotropic_dirs(rk, n_face)
    comp = d_f[np.arange(n_face), ax]
    flip = comp * sgn > 0.0                          # pointing out of the box
    d_f[flip, ax[flip]] = -comp[flip]
    origins = np.ascontiguousarray(np.concatenate([o_in, o_f]))
    dirs = np.ascontiguousarray(np.concatenate([d_in, d_f]))
    return Workload("clumpy", box, sites, density, origins, dirs, 1.0,
                    dict(seed=seed, M=M, N=N, n_clumps=n_clumps, n_from_clumps=n_in))


# --------------------------------------------------------------------------
# Tensor-product lattices (closed-form cuboid cells)
# --------------------------------------------------------------------------

def tensor_lattice(xs, ys, zs, box, N: int = 1000, seed: int = SEED_BASE + 100) -> Workload:
    """Sites {x_i} x {y_j} x {z_k}; site index (i*ny + j)*nz + k. Every cell is a
    cuboid bounded by the midpoints of consecutive coordinates and the box."""
    xs, ys, zs = (np.asarray(v, dtype=np.float64) for v in (xs, ys, zs))
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    sites = np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    box = np.asarray(box, dtype=np.float64)
    rs, rd, ro, rk = _streams(seed)
    density = rd.random(sites.shape[0])
    origins = uniform_in_box(ro, N, box)
    dirs = isotropic_dirs(rk, N)
    return Workload("tensor_lattice", box, sites, density, origins, dirs, 1.0,
                    dict(seed=seed, shape=(len(xs), len(ys), len(zs)), xs=xs, ys=ys, zs=zs))


def cubic_lattice(n: int = 8, N: int = 1000, seed: int = SEED_BASE + 101) -> Workload:
    """Dyadic cubic lattice: box [0,n]^3, sites at integer + 1/2; every cell is a
    unit cube and every bisector plane is exactly representable."""
    c = np.arange(n, dtype=np.float64) + 0.5
    return tensor_lattice(c, c, c, [0, 0, 0, n, n, n], N=N, seed=seed)


def random_tensor_lattice(shape=(5, 7, 4), N: int = 1000, seed: int = SEED_BASE + 102) -> Workload:
    rs = np.random.default_rng(seed)
    box = np.array([-1.0, -2.0, -0.5, 1.5, 1.0, 0.5])
    axes = []
    for a, n in enumerate(shape):
        lo, hi = box[a], box[a + 3]
        axes.append(np.sort(lo + (hi - lo) * rs.random(n)))
    return tensor_lattice(*axes, box, N=N, seed=seed + 1)


# --------------------------------------------------------------------------
# Serving mix (configuration 4)
# --------------------------------------------------------------------------

def serving_grids(seed: int = SEED_BASE + 4, scale: float = 1.0):
    """The three resident grids of the serving mix: 10^4 sites shaped like the
    uniform cube, 10^5 like the exponential disc, 10^6 like the flared disc."""
    g0 = uniform_cube(M=int(10_000 * scale), N=1, seed=seed)
    g1 = exp_disc(M=int(100_000 * scale), N=1, seed=seed + 10)
    g2 = flared_disc(M=int(1_000_000 * scale), N=2, seed=seed + 20)
    return [g0, g1, g2]


def serving_requests(n_req: int, grids, rate_hz: float, seed: int = SEED_BASE + 5,
                     lo: int = 256, hi: int = 65536):
    """Poisson arrivals (exponential gaps at ``rate_hz``), request sizes
    log-uniform in [lo, hi], grid chosen uniformly, accuracy class 50/50
    (0 = FP64, 1 = mixed). Rays are drawn the way each grid's workload draws
    them (uniform origins for the cube, site origins for the discs)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_req)
    t = np.cumsum(gaps) - gaps[0]
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n_req)).astype(np.int64)
    gid = rng.integers(0, len(grids), n_req)
    cls = rng.integers(0, 2, n_req)
    reqs = []
    for i in range(n_req):
        g = grids[gid[i]]
        n = int(sizes[i])
        if g.name == "uniform_cube":
            o = uniform_in_box(rng, n, g.box)
        else:
            o = np.ascontiguousarray(g.sites[rng.integers(0, g.M, n)])
        d = isotropic_dirs(rng, n)
        reqs.append(dict(t=float(t[i]), grid=int(gid[i]), mode=int(cls[i]), origins=o, dirs=d))
    return reqs


def grid_quality_points(box, n: int, seed: int = SEED_BASE + 6) -> np.ndarray:
    """n points uniform over the box: where the theoretical and the gridded
    density are compared (the grid-quality measure of Sect. 3.3)."""
    return uniform_in_box(np.random.default_rng(seed), n, box)


DENSITY_FIELDS = {
    "exp_disc": exp_disc_density,
    "flared_disc": flared_disc_density,
}


CONFIGS = {
    0: uniform_cube,
    1: exp_disc,
    2: flared_disc,
    3: clumpy,
}


def make_config(i: int, **kw) -> Workload:
    return CONFIGS[i](**kw)
