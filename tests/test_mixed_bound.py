"""The certified bounds of mixed mode, checked numerically on the CPU.

Mixed mode ranks each bisector plane by an FP32 crossing t and trusts the
ranking only where the intervals [t - err, t + err] separate the winner from
every other candidate; a step that is not separated is redone in FP64. The
ranking is exact only if every err really covers the distance from the FP32
t to the crossing that the FP64 step computes (Eq. 4, measured from the
current point). These tests restate the two FP32 formulas of the trace core
(FP32 records: the offset rounded to FP32; compact records: the offset as
integers against a power-of-two cell scale, with the quantisation term)
operation by operation in numpy float32 and check that claim on random and
adversarial planes: nearly parallel planes, neighbours far smaller than the
cell's largest offset, points far from the site, boxes far from the origin.
They also check the grazing band: a plane the FP32 test rejects as receding
(n.k <= -4d) must recede in FP64 too.

The FP32 operations are emulated with IEEE single rounding per operation; a
fused multiply-add is formed in double and rounded once to single (the
product of two singles is exact in double), and the hardware reciprocal is
taken at the worst of its one-ulp error on either side.
"""
import numpy as np

F = np.float32
U = 2.0 ** -24
EPS = 2.0 ** -20          # the default eps of the bound
Q_SHIFT = 19              # compact records: |q| <= 2^19 in the cell's units


def fma(a, b, c):
    return (np.float64(a) * np.float64(b) + np.float64(c)).astype(F)


def rcp_worst(den):
    """1/den rounded, then moved one ulp either way (the hardware reciprocal's
    error): both choices are returned."""
    r = (1.0 / den.astype(np.float64)).astype(F)
    return np.nextafter(r, F(np.inf)), np.nextafter(r, F(-np.inf))


def cross64(pj, pm, r0, k):
    """The FP64 crossing of the trace's FP64 step (no fused operations):
    n = pj - pm, s = n.((pj + pm)/2 - r0) / (n.k), and n.k."""
    n = pj - pm
    den = n[:, 0] * k[:, 0] + n[:, 1] * k[:, 1] + n[:, 2] * k[:, 2]
    w = 0.5 * (pj + pm) - r0
    num = n[:, 0] * w[:, 0] + n[:, 1] * w[:, 1] + n[:, 2] * w[:, 2]
    return num / den, den


def planes(rng, n, far=0.0, tiny=False, graze=False):
    """n planes: site pm, neighbour pj, ray origin r0 and direction k, and
    the current distance s_c along the ray (the current point inside or near
    the cell)."""
    scale = 10.0 ** rng.uniform(-3, 1, n)                     # cell sizes
    pm = far + rng.uniform(-100, 100, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    mag = scale * rng.uniform(0.3, 1.0, n)
    if tiny:   # neighbours far smaller than the cell's largest offset
        mag = mag * 10.0 ** rng.uniform(-7, -3, n)
    pj = pm + d * mag[:, None]
    k = rng.normal(size=(n, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    if graze:   # nearly parallel to the plane
        k = k - (k * d).sum(1, keepdims=True) * d
        k /= np.linalg.norm(k, axis=1, keepdims=True)
        tilt = 10.0 ** rng.uniform(-9, -3, n) * rng.choice([-1.0, 1.0], n)
        k = k + tilt[:, None] * d
        k /= np.linalg.norm(k, axis=1, keepdims=True)
    q = pm + rng.normal(size=(n, 3)) * scale[:, None] * rng.uniform(0.0, 2.0, n)[:, None]
    s_c = rng.uniform(0.0, 3.0, n) * scale
    r0 = q - s_c[:, None] * k
    return pm, pj, r0, k, s_c, scale


def e_abs_of(pm, pj, r0):
    """2^-48 times twice the largest coordinate plus the diagonal, per plane
    (the trace takes the box's; the points' own extent stands in here)."""
    pts = np.stack([pm, pj, r0], axis=1)
    cmax = np.abs(pts).max(axis=(1, 2))
    diag = np.linalg.norm(pts.max(axis=1) - pts.min(axis=1), axis=1)
    return 3.552713678800501e-15 * (2.0 * cmax + diag)


def fp32_bound(pm, pj, r0, k, s_c, e_abs):
    """The FP32-record crossing and bound: offsets rounded once to FP32."""
    nx, ny, nz = ((pj - pm).astype(F)).T
    q64 = (r0 + s_c[:, None] * k) - pm
    qx, qy, qz = q64.astype(F).T
    kx, ky, kz = k.astype(F).T
    c = F(3.0) * F(EPS)
    a = fma(c, np.sqrt(qx * qx + qy * qy + qz * qz), e_abs.astype(F))
    den = fma(nx, kx, fma(ny, ky, nz * kz))
    wx, wy, wz = fma(F(0.5), nx, -qx), fma(F(0.5), ny, -qy), fma(F(0.5), nz, -qz)
    num = fma(nx, wx, fma(ny, wy, nz * wz))
    n1 = np.abs(nx) + np.abs(ny) + np.abs(nz)
    d4 = fma(F(32.0 * U), n1, F(1.17549435e-38))
    out = []
    for rc in rcp_worst(den):
        t = num * rc
        err = (n1 * rc) * fma(c, np.abs(t), a)
        out.append((t, err))
    return out, den, d4, 1.0


def compact_bound(pm, pj, r0, k, s_c, e_abs, largest):
    """The compact-record crossing and bound in the cell's units: offsets as
    rint(offset * 2^(19 - E)), E the exponent above the cell's largest
    offset component."""
    E = np.floor(np.log2(largest)).astype(int) + 1
    qs = np.ldexp(1.0, Q_SHIFT - E)
    nint = np.rint((pj - pm) * qs[:, None])
    assert np.all(np.abs(nint) <= 2 ** Q_SHIFT)
    nx, ny, nz = nint.astype(F).T                              # exact
    q64 = ((r0 + s_c[:, None] * k) - pm) * qs[:, None]
    qx, qy, qz = q64.astype(F).T
    kx, ky, kz = k.astype(F).T
    e_abs_s = (e_abs * qs).astype(F)
    c = F(3.0) * F(EPS)
    a = fma(c, np.sqrt(qx * qx + qy * qy + qz * qz), e_abs_s)
    aq = F(0.6667) * (np.abs(qx) + np.abs(qy) + np.abs(qz) + F(0.75))
    den = fma(nx, kx, fma(ny, ky, nz * kz))
    wx, wy, wz = fma(F(0.5), nx, -qx), fma(F(0.5), ny, -qy), fma(F(0.5), nz, -qz)
    num = fma(nx, wx, fma(ny, wy, nz * wz))
    n1 = np.abs(nx) + np.abs(ny) + np.abs(nz)
    d4 = fma(F(32.0 * U), n1, F(3.5))
    out = []
    for rc in rcp_worst(den):
        t = num * rc
        e = (n1 * rc) * fma(c, np.abs(t), a)
        err = fma(F(1.34), e, rc * fma(F(1.16), np.abs(t), fma(F(0.6667), n1, aq)))
        out.append((t, err))
    return out, den, d4, qs


def check(res, pm, pj, r0, k, s_c):
    """Assert the bound on every certified plane; return their number and
    the largest error seen as a fraction of its bound."""
    out, den32, d4, qs = res
    s64, den64 = cross64(pj, pm, r0, k)
    want = (s64 - s_c) * qs                  # the FP64 crossing from the current point, in the same units
    pos = den32 > d4
    certified, worst = 0, 0.0
    for t, err in out:
        ok = np.isfinite(t) & np.isfinite(err)
        sel = pos & ok
        gap = np.abs(t.astype(np.float64) - want)
        bad = sel & (gap > err.astype(np.float64))
        assert not bad.any(), (int(bad.sum()), float((gap[bad] / err[bad]).max()))
        certified += int(sel.sum())
        if sel.any():
            worst = max(worst, float((gap[sel] / err[sel]).max()))
    # the grazing band: planes taken as receding in FP32 recede in FP64
    recede = den32 <= -d4
    assert np.all(den64[recede] < 0.0)
    # and planes taken as approached are approached in FP64
    assert np.all(den64[pos] > 0.0)
    return certified, worst


@np.errstate(all="ignore")
def test_fp32_record_bound():
    rng = np.random.default_rng(20131854)
    n_cert, worst = 0, 0.0
    for far, graze in ((0.0, False), (1e6, False), (0.0, True), (1e6, True)):
        p = planes(rng, 200_000, far=far, graze=graze)
        pm, pj, r0, k, s_c, _ = p
        c, w = check(fp32_bound(pm, pj, r0, k, s_c, e_abs_of(pm, pj, r0)), pm, pj, r0, k, s_c)
        n_cert, worst = n_cert + c, max(worst, w)
    assert n_cert > 500_000
    assert worst > 0.01   # the bound is not vacuous (about 15 times the largest error seen)


@np.errstate(all="ignore")
def test_compact_record_bound():
    rng = np.random.default_rng(20131855)
    n_cert, worst = 0, 0.0
    for far, tiny, graze in ((0.0, False, False), (1e6, False, False), (0.0, True, False), (0.0, False, True),
                             (1e6, True, True)):
        pm, pj, r0, k, s_c, scale = planes(rng, 200_000, far=far, tiny=tiny, graze=graze)
        largest = np.maximum(np.abs(pj - pm).max(axis=1), scale)   # the cell's largest offset component
        res = compact_bound(pm, pj, r0, k, s_c, e_abs_of(pm, pj, r0), largest)
        c, w = check(res, pm, pj, r0, k, s_c)
        n_cert, worst = n_cert + c, max(worst, w)
    assert n_cert > 400_000
    assert worst > 0.2    # the quantisation term is close to what rounding the offsets can do


@np.errstate(all="ignore")
def test_compact_bound_fails_without_the_quantisation_term():
    """The quantisation term is needed: with the FP32-record bound alone,
    some compact-record crossings fall outside their intervals (a planted
    omission that the check above must catch)."""
    rng = np.random.default_rng(7)
    pm, pj, r0, k, s_c, scale = planes(rng, 200_000)
    largest = np.maximum(np.abs(pj - pm).max(axis=1), scale)
    out, den32, d4, qs = compact_bound(pm, pj, r0, k, s_c, e_abs_of(pm, pj, r0), largest)
    # the FP32 bound alone: err = e (no 1.34 factor, no quantisation term)
    s64, _ = cross64(pj, pm, r0, k)
    want = (s64 - s_c) * qs
    t, _ = out[0]
    nx, ny, nz = np.rint((pj - pm) * qs[:, None]).astype(F).T
    n1 = np.abs(nx) + np.abs(ny) + np.abs(nz)
    q64 = ((r0 + s_c[:, None] * k) - pm) * qs[:, None]
    qn = np.linalg.norm(q64, axis=1)
    e_only = n1 / den32 * (3 * EPS * (np.abs(t) + qn) + e_abs_of(pm, pj, r0) * qs)
    pos = den32 > d4
    assert np.any(pos & (np.abs(t - want) > e_only))
