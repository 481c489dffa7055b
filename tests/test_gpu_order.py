"""The processing order of vor_order_rays, checked element by element.

vor_order_rays puts rays in a coherent order: by the Hilbert index of the
origin, then of the direction (a stable radix sort of each 30-bit key), and,
from 2^17 rays on, cut into 8 parts with the rays of each part grouped by
chord length, longest first (16 groups below 2^22 rays, 8 from there on). The order changes no result (the parity tests
show that); these tests check that it is the order those keys define, which
pins the radix sort (every digit, stability, tiles of 1024 keys below 2^22
keys and of 4096 above, rows of more than 2048 tiles, the ragged tail) and
the chord groups. The keys are restated here in numpy from their
definition: coordinates quantised to 10 bits over the box (origins) or over
[-1, 1] (unit directions), the Hilbert index by Skilling's transform
(J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004),
and the chord as the distance to the wall the ray heads for over the box
diagonal, as an 8-bit key smallest for the longest chords.
"""
import numpy as np
import pytest

from paper_1310_1854_amd import workloads as W

pytestmark = pytest.mark.gpu

BITS = 10
PARTS = 8
BINS_SMALL, BINS, BINS_SMALL_MAX_RAYS = 16, 8, 1 << 22
CHORD_MIN_RAYS = 1 << 17
ORDER_MIN_RAYS = 1 << 14


@pytest.fixture(scope="module")
def vrt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1310_1854_amd import vrt as v
    v.load()
    return v


def hilbert(x, y, z):
    """Skilling's axes-to-transpose, then the transpose's bits interleaved
    (x first), for uint32 arrays of BITS-bit coordinates."""
    X = [x.astype(np.uint32).copy(), y.astype(np.uint32).copy(), z.astype(np.uint32).copy()]
    Q = np.uint32(1 << (BITS - 1))
    while Q > 1:
        P = np.uint32(Q - 1)
        for i in range(3):
            hit = (X[i] & Q) != 0
            t = (X[0] ^ X[i]) & P
            X[0] = np.where(hit, X[0] ^ P, X[0] ^ t)
            if i:
                X[i] = np.where(hit, X[i], X[i] ^ t)
        Q = np.uint32(Q >> 1)
    X[1] ^= X[0]
    X[2] ^= X[1]
    t = np.zeros_like(X[0])
    Q = np.uint32(1 << (BITS - 1))
    while Q > 1:
        t = np.where((X[2] & Q) != 0, t ^ np.uint32(Q - 1), t)
        Q = np.uint32(Q >> 1)
    X = [a ^ t for a in X]
    key = np.zeros_like(X[0])
    for b in range(BITS - 1, -1, -1):
        key = (key << np.uint32(3)) | (((X[0] >> np.uint32(b)) & 1) << np.uint32(2)) \
            | (((X[1] >> np.uint32(b)) & 1) << np.uint32(1)) | ((X[2] >> np.uint32(b)) & 1)
    return key


def quant(f):
    return np.where(f > 0.0, np.minimum(f, 1023.0), 0.0).astype(np.uint32)


def expected_order(origins, dirs, box):
    lo, hi = np.asarray(box[:3], float), np.asarray(box[3:], float)
    N = origins.shape[0]
    kn = np.sqrt(dirs[:, 0] * dirs[:, 0] + dirs[:, 1] * dirs[:, 1] + dirs[:, 2] * dirs[:, 2])
    kn = np.where((kn > 0.0) & np.isfinite(kn), kn, 1.0)
    scale = 1024.0 / (hi - lo)
    qo, qd, L = [], [], np.full(N, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(3):
            ka = dirs[:, a] / kn
            qo.append(quant((origins[:, a] - lo[a]) * scale[a]))
            qd.append(quant((ka + 1.0) * 512.0))
            L = np.where(ka > 0.0, np.fmin(L, (hi[a] - origins[:, a]) / ka), L)
            L = np.where(ka < 0.0, np.fmin(L, (lo[a] - origins[:, a]) / ka), L)
    okey = hilbert(*qo)
    dkey = hilbert(*qd)
    coherent = np.lexsort((np.arange(N), dkey, okey))          # origin, then direction, then index
    if N < CHORD_MIN_RAYS:
        return coherent
    d2 = 0.0
    for a in range(3):
        d2 += (hi[a] - lo[a]) * (hi[a] - lo[a])
    diag = np.sqrt(d2)
    frac = np.where((L > 0.0) & (L < 1e300), np.fmin(L / diag, 1.0), 0.0)
    ckey = ((1.0 - frac) * 255.0 + 0.5).astype(np.int64)
    cnt = np.bincount(ckey, minlength=256)
    before = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    bins = BINS_SMALL if N < BINS_SMALL_MAX_RAYS else BINS
    bin_of = ((before + cnt // 2) * bins) // N                   # the middle rank of each key's run
    r = np.arange(N)
    final = (r * PARTS) // N * bins + bin_of[ckey[coherent]]
    return coherent[np.argsort(final, kind="stable")]


def gpu_order(vrt, grid, origins, dirs):
    import torch
    N = origins.shape[0]
    o = torch.as_tensor(origins, device="cuda")
    d = torch.as_tensor(dirs, device="cuda")
    order = torch.empty(N, dtype=torch.int32, device="cuda")
    ws = torch.empty(int(vrt.load().vor_order_workspace_bytes(N)), dtype=torch.uint8, device="cuda")
    vrt.order_rays(grid, o, d, order, ws)
    return order.cpu().numpy()


@pytest.mark.parametrize("N,seed", [(ORDER_MIN_RAYS, 1), (CHORD_MIN_RAYS - 1, 2), (300_001, 3), (3_000_000, 5)])
def test_order_is_the_key_order(vrt, N, seed):
    w = W.flared_disc(M=20_000, N=N, seed=seed)
    grid = vrt.build_grid(w.sites, w.box)
    got = gpu_order(vrt, grid, w.origins, w.dirs)
    want = expected_order(w.origins, w.dirs, w.box)
    assert np.array_equal(got, want)


def test_order_of_many_rays_with_shared_keys(vrt):
    """9x10^6 rays (more than 2048 sort tiles per digit row) with many equal
    keys: half the rays from one point, directions from a coarse set, so the
    sort's stability decides most of the order."""
    rng = np.random.default_rng(4)
    w = W.flared_disc(M=5_000, N=16, seed=4)
    lo, hi = np.asarray(w.box[:3]), np.asarray(w.box[3:])
    N = 9_000_000
    origins = lo + (hi - lo) * rng.random((N, 3))
    origins[: N // 2] = 0.5 * (lo + hi)
    dirs = rng.integers(-3, 4, size=(N, 3)).astype(np.float64)
    dirs[np.all(dirs == 0, axis=1)] = (1.0, 0.0, 0.0)
    grid = vrt.build_grid(w.sites, w.box)
    got = gpu_order(vrt, grid, origins, dirs)
    want = expected_order(origins, dirs, w.box)
    assert np.array_equal(got, want)
