/*
 * voronoi_rt.h -- C ABI of libvoronoi_rt, straight paths through a
 * box-clipped 3D Voronoi grid on an AMD Instinct MI355X (gfx950).
 *
 * The operations follow Camps, Baes & Saftly, "Using 3D Voronoi grids in
 * radiative transfer simulations": a setup phase that keeps the domain box,
 * the sites and per-site neighbour lists (Sect. 2.2, setup items 1-3), the
 * cell-location function C(r) (Sect. 2.3), and the path loop that moves
 * from cell to cell through the nearest bisector plane (Sect. 2.2, Eqs. 1-5).
 *
 * Conventions shared by every call:
 *  - Every entry point returns a vor_status and never throws.
 *  - Pointers documented as "device" are HIP device (or managed) memory on
 *    the current device; "host" pointers are ordinary CPU memory.
 *  - The caller owns every input and output buffer. A vor_grid owns its own
 *    device arrays until vor_grid_free.
 *  - Cells are identified by the 0-based index of their site in the caller's
 *    site array ("user order"). Box walls are negative: -1 xmin, -2 xmax,
 *    -3 ymin, -4 ymax, -5 zmin, -6 zmax.
 *  - A box is 6 doubles {xmin, ymin, zmin, xmax, ymax, zmax}; it is closed.
 *  - Point arrays are N x 3 row-major doubles (x, y, z per point).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it in order. vor_build_grid synchronises the stream
 *    before it returns; vor_locate and vor_trace do not synchronise and
 *    allocate nothing, so their results are ready when the stream is.
 *  - Argument errors are reported before any device work is enqueued.
 */
#ifndef VORONOI_RT_H
#define VORONOI_RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VOR_OK = 0,
    VOR_EINVAL = 1,     /* a bad argument: NULL pointer, negative size, empty box, ... */
    VOR_EDUP = 2,       /* two sites coincide */
    VOR_EOUTSIDE = 3,   /* a site lies outside the box or is not finite */
    VOR_ENOMEM = 4,     /* a device allocation failed */
    VOR_EDEVICE = 5,    /* a HIP runtime call or kernel launch failed */
    VOR_ECAPACITY = 6,  /* a cell needs more faces than the builder's fixed capacity, the neighbour
                           tables exceed 2^31 16-byte slots, or vor_trace_noalloc got more rays than
                           VOR_NOALLOC_MAX_RAYS */
    VOR_EBUDGET = 7,    /* a serving request exceeds the memory budget */
    VOR_ETIMEOUT = 8    /* a wait ran out of time; the request is still pending */
} vor_status;

/* Per-ray status written by vor_trace. */
enum {
    VOR_RAY_OK = 0,
    VOR_RAY_OUTSIDE = 1,    /* origin outside the closed box: no path, cell -1 */
    VOR_RAY_BADDIR = 2,     /* direction zero or not finite */
    VOR_RAY_STEPLIMIT = 3,  /* the path needed more steps than max_steps */
    VOR_RAY_OVERFLOW = 4    /* more segments than the ray's output capacity; counted, not stored */
};

enum {
    VOR_WALL_XMIN = -1, VOR_WALL_XMAX = -2, VOR_WALL_YMIN = -3,
    VOR_WALL_YMAX = -4, VOR_WALL_ZMIN = -5, VOR_WALL_ZMAX = -6
};

/* Arithmetic of the exit-point search. */
enum {
    VOR_MODE_FP64 = 0,  /* every bisector crossing in FP64 */
    VOR_MODE_MIXED = 1  /* FP32 plane tests, FP64 re-decision of close calls and FP64 winner */
};

/* Or'ed into vor_server_submit's mode: the request's densities are those
 * bound to its grid by vor_grid_bind_density (its density argument must be
 * NULL). */
#define VOR_SERVE_GRID_DENSITY 0x100

typedef struct vor_grid vor_grid;

/* Segments per spill chunk (see vor_trace_out). */
#define VOR_SPILL_CHUNK 64

/* Control words of a trace (vor_trace_out.work). */
#define VOR_WORK_WORDS 16

/* Options of vor_build_grid; zero-initialised fields take the defaults. */
typedef struct {
    double bucket_occupancy;  /* mean sites per bucket of the uniform site grid (default 2) */
    int32_t block_lists;      /* 1: also build the locate structure of Sect. 2.3 (blocks of a regular grid,
                                 each listing the cells whose bounding box overlaps it) and keep the cells'
                                 bounding boxes, for vor_locate_blocks and vor_grid_bboxes; 0: not */
    double block_occupancy;   /* with block_lists: about M / block_occupancy blocks (default 0.25) */
    int32_t record_layout;    /* the neighbour records that mixed-mode traces read (results are the same either
                                 way): VOR_RECORDS_AUTO (0, default: compact when the FP32 table would exceed
                                 512 MiB, i.e. would not stay in the last-level cache), VOR_RECORDS_FP32 (12-byte
                                 records: each neighbour offset p_j - p_m rounded to FP32) or VOR_RECORDS_COMPACT
                                 (8-byte records: the offset as three 21-bit integers against a power-of-two
                                 scale per cell) */
} vor_build_opts;

enum { VOR_RECORDS_AUTO = 0, VOR_RECORDS_FP32 = 1, VOR_RECORDS_COMPACT = 2 };

/* Facts about a built grid, filled by vor_grid_get_info. */
typedef struct {
    int64_t n_sites;          /* M */
    int64_t nnz;              /* total site-neighbour entries (walls excluded) */
    int64_t nnz_with_walls;   /* entries of the vor_grid_neighbors export */
    int32_t max_row;          /* longest site-neighbour list */
    int32_t dims[3];          /* bucket grid */
    double box[6];
    double build_ms;          /* wall time of vor_build_grid */
    int64_t device_bytes;     /* device memory held by the grid */
    int32_t block_dims[3];    /* blocks of the Sect. 2.3 locate structure (0 if not built) */
    int64_t block_entries;    /* total length of its cell lists */
    int32_t record_layout;    /* VOR_RECORDS_FP32 or VOR_RECORDS_COMPACT, as built */
} vor_grid_info;

/* Device memory for a grid's arrays, e.g. from a framework's caching
 * allocator. alloc returns `bytes` bytes of device memory usable in work
 * ordered on `stream` (the stream passed to vor_build_grid), or NULL when it
 * has none (vor_build_grid then fails with VOR_ENOMEM); free takes back a
 * block alloc gave, with its size. Both are called on the calling host
 * thread only: alloc and free during vor_build_grid (free for its
 * temporaries, after the stream has synchronised), free again in
 * vor_grid_free (after the device has synchronised) for the grid's own
 * arrays. ctx is passed through. The struct is copied into the grid; the
 * functions and ctx must stay valid until vor_grid_free. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx, void *stream);
    void (*free)(void *ptr, size_t bytes, void *ctx, void *stream);
    void *ctx;
} vor_allocator;

/*
 * vor_build_grid -- setup phase of Sect. 2.2 (items 1-3): keeps the box and
 * the sites and derives each site's neighbour list. The neighbours of site i
 * are found by clipping the box with the bisector half-spaces of nearby
 * sites (Sect. 2.1: a cell is the set of points at least as close to its
 * site as to any other); candidates come from a uniform bucket grid in
 * rings of increasing distance and the search stops when no farther site
 * can cut the cell. Lists are symmetric and may hold degenerate contacts
 * (an edge or vertex shared with a cell), which never change a path.
 *   sites  device, M x 3, user order; read during the call only.
 *   M      number of sites, >= 1 and < 2^31.
 *   box    host, 6 doubles, xmin < xmax etc.; every site must lie inside.
 *   opts       host, may be NULL.
 *   allocator  host, may be NULL (hipMalloc and hipFree): where the grid's
 *              device memory comes from (see vor_allocator).
 *   out        host; receives the grid on VOR_OK, NULL otherwise.
 * Errors: VOR_EINVAL, VOR_EOUTSIDE (a site outside the box or not finite),
 * VOR_EDUP (coincident sites), VOR_ENOMEM, VOR_ECAPACITY, VOR_EDEVICE.
 * Synchronises `stream` before returning.
 */
vor_status vor_build_grid(const double *sites, int64_t M, const double *box,
                          const vor_build_opts *opts, const vor_allocator *allocator, void *stream,
                          vor_grid **out);

/* Releases every device array of the grid (synchronises the device first). NULL is a no-op. */
void vor_grid_free(vor_grid *grid);

/* Fills *info (host). */
vor_status vor_grid_get_info(const vor_grid *grid, vor_grid_info *info);

/*
 * vor_grid_volumes -- the volume of every clipped cell (Sect. 2.1: the box
 * cut by the bisector half-spaces), from the builder's own clipped
 * polyhedra: the sum over the faces of the cone volumes h * area / 3 from
 * the site. volume: device, M doubles, user order. Asynchronous on `stream`.
 */
vor_status vor_grid_volumes(const vor_grid *grid, double *volume, void *stream);

/*
 * vor_grid_bboxes -- the bounding box of every clipped cell (Sect. 2.3: from
 * its vertices, the cell being convex), as the builder computed it.
 *   bbox  device, M x 6 doubles {xmin, ymin, zmin, xmax, ymax, zmax}, user order.
 * VOR_EINVAL unless the grid was built with opts.block_lists = 1.
 * Asynchronous on `stream`.
 */
vor_status vor_grid_bboxes(const vor_grid *grid, double *bbox, void *stream);

/*
 * vor_grid_bind_density -- keeps an exact copy of a density field (the rho_m
 * of the optical depth, Sect. 2.2: tau = kappa * sum of rho_m l_m over the
 * segments) inside the grid, for traces that ask for it with
 * vor_trace_opts.grid_density = 1 (and server requests with
 * VOR_SERVE_GRID_DENSITY): beside each cell's site in its block, where a
 * mixed-mode step reads it with the cell's other data, and in the grid's
 * internal (spatial) order for FP64 mode, instead of from an array in user
 * order. The grid holds the room for both copies from its build.
 *   density  device, M doubles, user order; read during the call only. NULL
 *            removes the bound field.
 * Asynchronous on `stream`; allocates nothing. Changes the grid: traces
 * that overlap the call on another stream may see either field.
 */
vor_status vor_grid_bind_density(vor_grid *grid, const double *density, void *stream);

/*
 * vor_grid_neighbors -- the neighbour lists of Sect. 2.2 item 3 in CSR form,
 * user order, walls as negative codes (Sect. 2.2: walls are special
 * negative indices). Row i lists, in increasing order, the neighbour cells
 * of site i followed by its wall codes.
 *   row_ptr  device, M + 1 int64 (row i spans [row_ptr[i], row_ptr[i+1])).
 *   col      device, info.nnz_with_walls int32.
 * Asynchronous on `stream`.
 */
vor_status vor_grid_neighbors(const vor_grid *grid, int64_t *row_ptr, int32_t *col, void *stream);

/*
 * vor_locate -- the function C(r) of Sect. 2.3: for each point the index of
 * the cell containing it, i.e. of the nearest site (squared distances; equal
 * distances go to the lowest index), or -1 for a point outside the closed box
 * (step 1 there). Candidate sites come from the bucket grid in rings of
 * increasing distance until no farther bucket can hold a nearer site.
 *   pts   device, N x 3.     cell  device, N int32.    N >= 0.
 * Asynchronous on `stream`; allocates nothing.
 */
vor_status vor_locate(const vor_grid *grid, const double *pts, int64_t N, int32_t *cell, void *stream);

/*
 * vor_locate_blocks -- C(r) as Sect. 2.3 builds it: -1 outside the closed
 * box (step 1); else the block of the regular grid holding the point
 * (step 2), the cells listed for that block -- those whose bounding box,
 * widened by 1e-9 of its extent, overlaps it (step 3) -- and the nearest of
 * their sites by squared distance, equal distances going to the lowest index
 * (step 4). Same result as vor_locate.
 *   pts   device, N x 3.     cell  device, N int32.    N >= 0.
 * VOR_EINVAL unless the grid was built with opts.block_lists = 1.
 * Asynchronous on `stream`; allocates nothing.
 */
vor_status vor_locate_blocks(const vor_grid *grid, const double *pts, int64_t N, int32_t *cell, void *stream);

/* Options of vor_trace; zero-initialised fields take the defaults. */
typedef struct {
    int32_t mode;           /* VOR_MODE_FP64 (default) or VOR_MODE_MIXED */
    int32_t max_steps;      /* per-ray cap on cell moves; 0 = M + 16 */
    double eps_mix;         /* mixed mode: relative rounding allowance of the FP32 crossing bound; 0 = 2^-20,
                               else in [2^-20, 0.25] (larger values only redo more steps in FP64) */
    int32_t persistent;     /* 1: persistent kernel whose waves refill finished lanes from a work queue */
    int32_t start_given;    /* 1: out->start_cell already holds the start cells of these rays, left there by
                               an earlier call on the same grid with the same origins (another density,
                               kappa or mode); the start-cell pass is skipped */
    int32_t enter;          /* 1: a ray whose origin lies outside the box (Sect. 2.2 notes the method extends
                               to such rays) starts where it enters the box: s0 = the largest over the axes of
                               the distance to the near wall; distances stay measured from the origin, the
                               start cell is C(r0 + s0 k); a ray that misses the box (s0 >= L) or has a
                               non-finite origin gets VOR_RAY_OUTSIDE. 0: every origin outside the box is
                               VOR_RAY_OUTSIDE */
    int32_t grid_density;   /* 1: the densities are those bound to the grid by vor_grid_bind_density (the
                               density argument must then be NULL); tau is the same as with that field
                               passed as the density argument. VOR_EINVAL if none is bound */
    double eps_fb;          /* the no-exit fallback's advance (Sect. 2.2: move the point a small distance
                               along the ray, then locate it again), a distance; 0 = 1e-12 times the box
                               diagonal. The advance is not part of any segment, so such a path's lengths
                               sum to L - n_fallback * eps_fb. VOR_EINVAL if negative or not finite */
} vor_trace_opts;

/* Outputs of vor_trace. All pointers are device memory; tau and n_seg are required. */
typedef struct {
    double *tau;            /* [N] optical depth kappa * sum(rho_m * l_m) in path order */
    int32_t *n_seg;         /* [N] number of segments of the full path (also past capacity) */
    uint8_t *status;        /* [N] VOR_RAY_*; may be NULL */
    int32_t *n_fallback;    /* [N] no-exit fallbacks taken (Sect. 2.2); may be NULL */
    int32_t *seg_cell;      /* segment cells (user order); NULL = tau-only */
    double *seg_len;        /* segment lengths; NULL with seg_cell NULL */
    int64_t seg_stride;     /* > 0: ray i owns slots [i*seg_stride, (i+1)*seg_stride) */
    const int64_t *ray_off; /* seg_stride == 0: ray i owns [ray_off[i], ray_off[i+1]) */
    unsigned long long *counters; /* [8] accumulated: segments, fallbacks, FP64 re-decisions, steps,
                                     neighbour records read, wave iterations and refills of the persistent
                                     kernel (steps / (64 x iterations) is its lane utilisation), 1 reserved;
                                     may be NULL */
    int64_t *work;          /* [VOR_WORK_WORDS] device control words, required for persistent mode and spill;
                               zeroed by the call. work[2] ends as the number of rays whose path continued
                               past its window; the others are the work queues and chunk counter. */
    /* Spill (stride mode only, all NULL to disable): a ray whose path is
     * longer than seg_stride keeps its first seg_stride segments in its
     * window and continues in a chain of chunks of VOR_SPILL_CHUNK slots in
     * spill_cell/spill_len: spill_first[i] is the ray's first chunk (-1 if
     * none), spill_next[c] the chunk after chunk c (-1 at the end). Chunks
     * are handed out as paths grow, in one pass. If the chunks run out the
     * ray's status is VOR_RAY_OVERFLOW (count and tau stay complete).
     * work[1] ends as the number of chunks asked for. */
    int64_t *spill_first;   /* [N] */
    int32_t *spill_next;    /* [spill_chunks] */
    int32_t *spill_cell;    /* [spill_chunks * VOR_SPILL_CHUNK] */
    double *spill_len;      /* [spill_chunks * VOR_SPILL_CHUNK] */
    int64_t spill_chunks;
    const int32_t *ray_order; /* optional [N]: lane i traces ray ray_order[i] (a permutation, e.g. from
                                 vor_order_rays); outputs stay indexed by ray */
    int32_t *start_cell;    /* optional [N] scratch: when set, the start cells C(r0) of all rays are located
                               in a pass of their own before the traversal (faster, mostly with the
                               persistent kernel) and left here (internal cell indices, -1 for rays
                               without a path) for reuse through opts.start_given */
    /* Transport along the paths (optional; the photon-package transport that the paths serve, Sect. 3.4).
     * Interaction points: with tau_k the optical depth after the k-th segment (summed as above), a path
     * stops in the first cell m_k with kappa rho_m > 0 and tau_k >= tau_stop[i], at distance
     * s_{k-1} + (tau_stop - tau_{k-1}) / (kappa rho_m) from the origin; its last segment is cut there,
     * tau and n_seg describe the cut path. tau_stop <= 0 stops at the origin, in the start cell, before
     * any segment. Tallies: per cell (user order), accumulated over the calls (never zeroed here),
     *   tally_len[m] += w l,   tally_abs[m] += w exp(-tau before the segment) (1 - exp(-kappa rho_m l))
     * for every segment (m, l) of the (cut) path, w = weight[i] or 1; the absorbed fractions of one path
     * sum to w (1 - exp(-tau)). Floating-point atomics: the order of the sums is not fixed. */
    const double *tau_stop; /* [N] or NULL: the optical depth at which each path stops (e.g. -ln u) */
    int32_t *stop_cell;     /* [N], required with tau_stop: cell of the interaction point (user index),
                               -1 when the path reaches the wall first or has no path */
    double *stop_s;         /* [N] or NULL, with tau_stop only: distance of the interaction point from the
                               origin; the chord L when the path reached the wall */
    double *tally_len;      /* [M] or NULL */
    double *tally_abs;      /* [M] or NULL */
    const double *weight;   /* [N] or NULL (weights 1); only with a tally */
} vor_trace_out;

/*
 * vor_trace -- straight paths (Sect. 2.2). Each ray starts at origins[i]
 * with direction dirs[i] (normalised here in FP64) and ends where it leaves
 * the box (Eq. 5 on every axis). The start cell is C(r0) (Sect. 2.3). Each
 * step evaluates, for every neighbour j of the current cell m whose bisector
 * plane the ray approaches (n.k > 0, n = p_j - p_m, Eq. 1), the crossing
 * s_j = n.((p_j + p_m)/2 - r0)/(n.k) (Eqs. 2-4, measured from the origin) and
 * leaves the cell at the smallest one, or at the wall if that comes first.
 * Segments of zero length are not emitted. Segment i of a ray is
 * (seg_cell, seg_len) at slot base + i of the ray's window; cells are user
 * indices.
 *   origins, dirs  device, N x 3.    density  device, M doubles (user order), or NULL (tau = 0).
 *   kappa          multiplies tau.   opts     host, may be NULL.
 *   out            host struct of device pointers.
 * VOR_MODE_MIXED ranks the planes in FP32 with a certified bound on each
 * crossing's rounding error and decides in FP64 whenever the bounds do not
 * separate the winner, so its results equal VOR_MODE_FP64's bit for bit.
 * Asynchronous on `stream`; allocates nothing. Per-ray problems are reported
 * in out->status, not as a return code; VOR_EINVAL for inconsistent
 * pointers, an option out of range, or mixed mode on a box with a
 * coordinate of magnitude 1e30 or more.
 */
vor_status vor_trace(const vor_grid *grid, const double *origins, const double *dirs, int64_t N,
                     const double *density, double kappa, const vor_trace_opts *opts,
                     const vor_trace_out *out, void *stream);

/* Rays per vor_trace_noalloc call. */
#define VOR_NOALLOC_MAX_RAYS (1 << 22)

/*
 * vor_trace_noalloc -- vor_trace for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation. The control words of the work queues and the spill
 * (vor_trace_out.work) and the start-cell scratch (vor_trace_out.start_cell)
 * come from a fixed array inside the library, 16 MiB per GPU (the control
 * words, then the start cells of up to VOR_NOALLOC_MAX_RAYS rays), which
 * each GPU the library runs on holds until the process ends; the caller
 * passes the inputs and outputs as to vor_trace, with out->work and
 * out->start_cell NULL and opts->start_given 0 (VOR_EINVAL otherwise).
 * Every call on a GPU uses that GPU's one array: calls ordered on one
 * stream are safe, calls that overlap on one GPU (other streams, other
 * threads) race and corrupt each other's paths. The first call on a device
 * looks up the array's address there (hipGetSymbolAddress) with that device
 * current. Allocates nothing.
 * Errors: those of vor_trace; VOR_ECAPACITY for N > VOR_NOALLOC_MAX_RAYS;
 * VOR_EDEVICE if the array cannot be reached.
 */
vor_status vor_trace_noalloc(const vor_grid *grid, const double *origins, const double *dirs, int64_t N,
                             const double *density, double kappa, const vor_trace_opts *opts,
                             const vor_trace_out *out, void *stream);

/*
 * vor_order_rays -- a processing order for a batch of rays that keeps
 * neighbouring lanes on neighbouring paths and starts long paths first: the
 * rays sorted by the Hilbert index of their origin (10 bits per axis over
 * the grid's box) and, among equal origins, of their direction, cut into 8
 * contiguous parts (the parts a persistent trace gives its XCDs), and inside
 * each part grouped by the length of their chord (the distance to the wall
 * they head for, Eq. 5 on every axis; 8 groups ranked over the batch), the
 * longest first, keeping that order within a group (batches of fewer than
 * 2^17 rays keep the first order alone; batches of fewer than 2^14 rays keep
 * their own order, the identity, as sorting them costs more than it saves).
 * Pass it as
 * vor_trace_out.ray_order; results do not depend on the order, only the
 * speed does.
 *   origins, dirs  device, N x 3.   order  device, N int32 (a permutation).
 *   workspace      device, at least vor_order_workspace_bytes(N) bytes.
 * Asynchronous; allocates nothing.
 */
vor_status vor_order_rays(const vor_grid *grid, const double *origins, const double *dirs, int64_t N,
                          int32_t *order, void *workspace, int64_t workspace_bytes, void *stream);
int64_t vor_order_workspace_bytes(int64_t N);

/*
 * vor_exclusive_scan -- offsets[0] = 0, offsets[i+1] = offsets[i] + counts[i]
 * (int64), e.g. to turn a tau-only pass's n_seg into ray_off for an exact
 * second pass. counts device N int32 (>= 0), offsets device N + 1 int64.
 * Asynchronous; allocates nothing (tile totals are staged inside offsets).
 */
vor_status vor_exclusive_scan(const int32_t *counts, int64_t N, int64_t *offsets, void *stream);

/*
 * vor_gather_paths -- whole paths as compact rows (Sect. 2.2: a path is every
 * cell it crosses, in order, to the wall) from a trace into segment windows:
 * ray i's segments -- the first min(n_seg[i], seg_stride) slots of its window,
 * then its chain of spill chunks -- go to [ray_off[i], ray_off[i] + n_seg[i])
 * of seg_cell / seg_len. With ray_off = vor_exclusive_scan(n_seg) this gives
 * the exact layout from one traversal, instead of a counting pass and a
 * second traversal into ray_off.
 *   n_seg, win_cell, win_len, spill_*   device, as the vor_trace_out of that
 *                  trace (seg_stride > 0) left them; the four spill arrays
 *                  are all NULL when the trace had no spill (then no ray may
 *                  have more than seg_stride segments);
 *   ray_off        device N + 1 int64; seg_cell / seg_len device, ray_off[N]
 *                  entries each, written.
 * A ray whose spill ran out (VOR_RAY_OVERFLOW) keeps only the segments that
 * were stored; the rest of its row is left unwritten. Argument errors:
 * VOR_EINVAL (N < 0, seg_stride <= 0, a missing array, some but not all
 * spill arrays). Asynchronous on `stream`; allocates nothing.
 */
vor_status vor_gather_paths(const int32_t *n_seg, int64_t N, const int32_t *win_cell, const double *win_len,
                            int64_t seg_stride, const int64_t *spill_first, const int32_t *spill_next,
                            const int32_t *spill_cell, const double *spill_len, const int64_t *ray_off,
                            int32_t *seg_cell, double *seg_len, void *stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of path requests over resident grids.
 *
 * A server keeps several built grids resident and accepts requests (a batch
 * of rays for one grid, in FP64 or mixed mode) from any host thread. A
 * request waits in a first-in-first-out queue until its output buffers fit
 * in the server's memory budget. Admitted requests are traced together by
 * persistent kernels on several streams: their rays are cut into chunks
 * that the waves take from a device work queue, refilling finished lanes,
 * and a later launch starts on the GPU as the blocks of an earlier one
 * retire. A request is complete as soon as its own rays are (the kernel
 * raises a flag in host memory), not when its launch ends. Every ray is
 * computed by the same code as vor_trace, so its result does not depend on
 * the other requests. Paths follow Sect. 2.2 as in vor_trace and are whole
 * (every cell to the wall): a ray's first seg_stride segments go to its
 * window and the rest to a chain of spill chunks of VOR_SPILL_CHUNK slots
 * from the request's own pool of spill_chunks chunks, taken as the path
 * grows. If the pool runs out for some ray, the request is traced again,
 * ahead of every waiting request, with exactly the chunks its segment counts
 * need (the paths are the same, so the second run cannot run out); its
 * results are those of that run. vor_server_copy_result returns the paths
 * as compact rows.
 * ------------------------------------------------------------------------- */
typedef struct vor_server vor_server;

typedef struct {
    int64_t completed;         /* requests finished */
    int64_t crossings;         /* segments emitted by finished launches (counted when a launch ends) */
    int64_t fp64_redecisions;  /* mixed-mode steps redone in FP64 */
    int64_t fallbacks;         /* no-exit fallbacks */
    int64_t launches;          /* kernel launches finished */
    int64_t running;           /* kernel launches in flight */
    int64_t waiting;           /* requests not yet admitted */
    int64_t budget_bytes;      /* output memory budget */
    int64_t used_bytes;        /* held by admitted, unreleased requests */
    double uptime_s;
    int64_t reruns;            /* requests traced a second time because their spill chunks ran out */
} vor_server_stats;

/* Create a server over n_grids built grids (host array of handles; the grids
 * must outlive the server) with a budget of device memory for request
 * outputs (allocated once here). Starts the scheduler thread. */
vor_status vor_server_create(const vor_grid *const *grids, int32_t n_grids, int64_t budget_bytes,
                             vor_server **out);

/* Queue a request: n rays (origins, dirs: device, n x 3) on grid `grid`,
 * density (device, that grid's M sites, user order; may be NULL), mode
 * VOR_MODE_*, optionally or'ed with VOR_SERVE_GRID_DENSITY (then density
 * must be NULL and the grid must hold a bound density when the request is
 * submitted; rebinding it before the request is done is not allowed),
 * seg_stride segment slots per ray (0 = tau only) and a first pool of
 * spill_chunks chunks for the segments past the windows (0 with seg_stride
 * 0; a pool too small costs a second run of the request, not segments).
 * The request is traced only after the work enqueued on `stream` (the
 * submitter's stream, a hipStream_t; NULL = the null stream) before this
 * call, so inputs still being written there are waited for. The inputs are
 * borrowed until the request is done. *req_id receives its handle.
 * VOR_EINVAL for a bad argument; VOR_EBUDGET if its outputs could never fit
 * in the budget (the first pool counts; a second run whose exact pool does
 * not fit ends the request with VOR_EBUDGET from vor_server_wait). */
vor_status vor_server_submit(vor_server *srv, int32_t grid, const double *origins, const double *dirs, int64_t n,
                             const double *density, double kappa, int32_t mode, int64_t seg_stride,
                             int64_t spill_chunks, void *stream, int64_t *req_id);

/* *done = 1 once the request's outputs are complete; they are then visible
 * to work on any stream and to copies to the host, even while the launch
 * that computed them is still running. */
vor_status vor_server_poll(vor_server *srv, int64_t req_id, int32_t *done);

/* Block until the request is done or timeout_s passes (VOR_ETIMEOUT).
 * Returns the request's own error once it is done (VOR_OK normally). */
vor_status vor_server_wait(vor_server *srv, int64_t req_id, double timeout_s);

/* Completion queue: *req_id receives the next request that has completed
 * (in completion order; each once, released ones skipped), waiting up to
 * timeout_s (VOR_ETIMEOUT, *req_id = 0, if none completes). */
vor_status vor_server_next_done(vor_server *srv, double timeout_s, int64_t *req_id);

/* Device pointers of a finished request's outputs (tau, n_seg, status; with
 * seg_stride the windows seg_cell/seg_len and the spill chain spill_first,
 * spill_next, spill_cell, spill_len, spill_chunks, laid out as in
 * vor_trace_out; server-owned until release) and its latency from
 * submission to completion in seconds. */
vor_status vor_server_result(vor_server *srv, int64_t req_id, vor_trace_out *out, double *latency_s);

/* Copy a finished request's outputs into caller buffers (device; any may be
 * NULL), asynchronously on `stream`: tau, n_seg, status (n each) and, for a
 * request with segments, the whole paths as compact rows -- ray i's
 * segments at [ray_off[i], ray_off[i] + n_seg[i]) of seg_cell/seg_len, with
 * ray_off (device, n + 1 int64) the exclusive scan of the request's counts
 * (vor_exclusive_scan of n_seg) and seg_cell/seg_len holding ray_off[n]
 * entries. A later vor_server_release waits for these copies: the memory
 * returns to the budget only once they have run. */
vor_status vor_server_copy_result(vor_server *srv, int64_t req_id, double *tau, int32_t *n_seg, uint8_t *status,
                                  const int64_t *ray_off, int32_t *seg_cell, double *seg_len, void *stream);

/* Return a finished request's outputs to the budget: at once, or, if copies
 * from vor_server_copy_result are still running, as soon as the last of them
 * has finished (the call itself does not wait). The device pointers of
 * vor_server_result must not be used after this call; work on them must
 * have completed before it. */
vor_status vor_server_release(vor_server *srv, int64_t req_id);

vor_status vor_server_get_stats(vor_server *srv, vor_server_stats *stats);

/* Finish in-flight work, stop the scheduler, free everything. NULL is a no-op. */
void vor_server_destroy(vor_server *srv);

/* Static description of a status code. */
const char *vor_status_str(vor_status s);

/* Library version string. */
const char *vor_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VORONOI_RT_H */
