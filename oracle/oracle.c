/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of what the straight-path method on
 * a box-clipped 3D Voronoi grid computes (Camps, Baes & Saftly, "Using 3D
 * Voronoi grids in radiative transfer simulations", Sect. 2). It shares no
 * code, header or table with the GPU library and is used only by the tests,
 * the smoke check and the CPU baseline of the benchmark.
 *
 * Every routine works from the definitions, by brute force over all sites:
 *   - a Voronoi cell is the set of points at least as close to its site as to
 *     any other site (Sect. 2.1), clipped by the domain box (Sect. 2.2);
 *   - the cell containing a point is the one whose site is nearest (Sect. 2.3);
 *   - a path is the ordered list of cells met by r0 + s k for s in [0, L),
 *     L being where the ray leaves the box (Sect. 2.2), each with the length
 *     travelled inside it.
 *
 * Readings where the paper is silent (documented beside each routine):
 *   ties at a cell boundary are resolved right-continuously (the cell nearest
 *   just after the crossing: largest k.p_j, then lowest index); a wall that
 *   ties a bisector plane ends the path; zero-length segments are never
 *   emitted; indices are 0-based; walls are -1..-6 = xmin,xmax,ymin,ymax,
 *   zmin,zmax; the optical depth is kappa * sum(rho_m * l_m) summed in path
 *   order.
 *
 * Box layout everywhere: {xmin, ymin, zmin, xmax, ymax, zmax}.
 * Per-ray status codes: 0 ok, 1 origin outside the box, 2 bad direction,
 * 3 step limit, 4 segment capacity exceeded (the path is still counted).
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 *        -fno-fast-math oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ST_OK 0
#define ST_OUTSIDE 1
#define ST_BADDIR 2
#define ST_STEPLIMIT 3
#define ST_OVERFLOW 4

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int inside_box(const double *box, const double *r)
{
    for (int a = 0; a < 3; ++a)
        if (!(r[a] >= box[a] && r[a] <= box[a + 3])) return 0;
    return 1;
}

static double dist2(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return dx * dx + dy * dy + dz * dz;
}

/*
 * oracle_locate -- the function C(r) of Sect. 2.3, steps 1 and 4, without the
 * block acceleration of steps 2-3 (which only narrows the candidate list):
 * -1 for a point outside the closed box, else the index of the nearest site
 * by squared distance; equal distances go to the lowest index.
 * If gap != NULL it receives, per point, the distance from the point to the
 * bisector plane of its two nearest sites, (d2^2 - d1^2) / (2 |p2 - p1|),
 * which measures how close the query is to a cell boundary (+inf if M < 2).
 */
int oracle_locate(const double *sites, int64_t M, const double *box,
                  const double *pts, int64_t N, int32_t *cell, double *gap)
{
    if (M <= 0) return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < N; ++q) {
        const double *r = pts + 3 * q;
        if (!inside_box(box, r)) {
            cell[q] = -1;
            if (gap) gap[q] = INFINITY;
            continue;
        }
        int64_t b1 = -1, b2 = -1;
        double d1 = INFINITY, d2 = INFINITY;
        for (int64_t j = 0; j < M; ++j) {
            double d = dist2(r, sites + 3 * j);
            if (d < d1) {
                d2 = d1; b2 = b1;
                d1 = d; b1 = j;
            } else if (d < d2) {
                d2 = d; b2 = j;
            }
        }
        cell[q] = (int32_t)b1;
        if (gap) {
            if (b2 < 0) gap[q] = INFINITY;
            else gap[q] = (d2 - d1) / (2.0 * sqrt(dist2(sites + 3 * b1, sites + 3 * b2)));
        }
    }
    return 0;
}

/*
 * oracle_trace -- one straight path per ray, brute force over all sites.
 *
 * The ray is r(s) = r0 + s k with k normalised here in FP64 (Sect. 2.2 asks
 * for a unit vector). L = min over axes with k_a != 0 of the distance to the
 * wall the ray heads for (Eq. 5 applied on every axis): the ray leaves the
 * box there.
 *
 * Start cell: the nearest site to r0 (Sect. 2.2: C(r0)); if several are
 * equally near, the one nearest just after s = 0, i.e. the largest k.p_j,
 * then the lowest index.
 *
 * Step (Sect. 2.2, Eqs. 1-4), with m the current cell and s_c the current
 * position along the ray: for every other site j whose bisector plane with m
 * is approached by the ray, n.k > 0 with n = p_j - p_m (Eq. 1), the crossing
 * parameter measured from the fixed origin r0 is
 *       s_j = n . ((p_j + p_m)/2 - r0) / (n . k)          (Eqs. 2-4)
 * and the cell is left at s* = min(L, min_j s_j). Planes with n.k <= 0 are
 * never crossed forwards (the ray moves away from them or along them) and
 * are skipped (the sign argument of Sect. 2.2). The segment (m, s* - s_c)
 * is emitted when its length is positive; tau accumulates kappa rho_m
 * times that length. If the wall attains s* (ties included) the path ends;
 * otherwise m becomes the winning site -- on equal s_j the one with the
 * largest n.k (nearest just after s*), then the lowest index -- and the
 * loop repeats. Every move goes to a site with a strictly larger k.p, so at
 * most M moves occur.
 *
 * Near-ties: at every step the two smallest candidates s(1) <= s(2) (the
 * wall included) are compared; a step with s(2) - s(1) <= eta * L counts in
 * n_near, and min_gap holds the smallest (s(2) - s(1)) / L over the path
 * together with the start-cell gap of oracle_locate divided by L.
 *
 * With enter != 0 a ray whose origin lies outside the box starts where it
 * enters the box: s0 = the largest over the axes of the distance to the
 * near wall (the walls it moves towards, Eq. 5 turned round); it misses the
 * box (status OUTSIDE) unless s0 < L. The start cell is then the nearest
 * site to r0 + s0 k, and crossings are still measured from r0.
 *
 * Outputs per ray (any may be NULL except nseg): segments at
 * seg_cell/seg_len[ray * cap + i] for i < cap, with seg_end the position
 * s* (from the origin) where each segment ends, nseg (true count even past
 * cap), tau, chord = L, status, n_near, min_gap, cell0 = start cell,
 * start_s = s0 (0 for origins inside the box).
 * Returns 0, or 1 on bad arguments.
 */
int oracle_trace(const double *sites, int64_t M, const double *box,
                 const double *rho, double kappa,
                 const double *origins, const double *dirs, int64_t N,
                 double eta, int64_t cap,
                 int32_t *seg_cell, double *seg_len, double *seg_end,
                 int32_t *nseg, double *tau, double *chord, int32_t *status,
                 int32_t *n_near, double *min_gap, int32_t *cell0,
                 int enter, double *start_s)
{
    if (M <= 0 || N < 0 || !nseg) return 1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ray = 0; ray < N; ++ray) {
        const double *r0 = origins + 3 * ray;
        double k[3] = {dirs[3 * ray], dirs[3 * ray + 1], dirs[3 * ray + 2]};
        double knorm = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
        int st = ST_OK;
        int32_t count = 0, near = 0;
        double t = 0.0, L = 0.0, gmin = INFINITY;
        int32_t start = -1;

        double s0 = 0.0;                     /* where the path starts, measured from r0 */
        const int outside = !inside_box(box, r0);
        if (!(knorm > 0.0) || !isfinite(knorm)) {
            st = ST_BADDIR;
        } else if (outside && (!enter || !isfinite(r0[0]) || !isfinite(r0[1]) || !isfinite(r0[2]))) {
            st = ST_OUTSIDE;
        }
        if (st == ST_OK) {
            for (int a = 0; a < 3; ++a) k[a] /= knorm;
            /* chord length to the box wall (Eq. 5 on each axis) */
            L = INFINITY;
            for (int a = 0; a < 3; ++a) {
                if (k[a] > 0.0) {
                    double s = (box[a + 3] - r0[a]) / k[a];
                    if (s < L) L = s;
                } else if (k[a] < 0.0) {
                    double s = (box[a] - r0[a]) / k[a];
                    if (s < L) L = s;
                }
            }
            if (outside) {
                /* a ray from outside enters the box where it has crossed the
                 * near wall of every axis (Sect. 2.2 notes the method extends
                 * to such rays); it misses the box if that is not before L */
                for (int a = 0; a < 3; ++a) {
                    if (k[a] > 0.0) {
                        double s = (box[a] - r0[a]) / k[a];
                        if (s > s0) s0 = s;
                    } else if (k[a] < 0.0) {
                        double s = (box[a + 3] - r0[a]) / k[a];
                        if (s > s0) s0 = s;
                    } else if (r0[a] < box[a] || r0[a] > box[a + 3]) {
                        s0 = INFINITY;
                    }
                }
                if (!(s0 < L)) {
                    st = ST_OUTSIDE;
                    L = 0.0;
                }
            }
        }
        if (st == ST_OK) {
            double q[3] = {r0[0], r0[1], r0[2]};   /* the start point */
            if (outside)
                for (int a = 0; a < 3; ++a) q[a] = r0[a] + s0 * k[a];
            /* start cell: nearest site, right-continuous tie rule */
            double d1 = INFINITY, d2 = INFINITY;
            int64_t m = -1, second = -1;
            for (int64_t j = 0; j < M; ++j) {
                double d = dist2(q, sites + 3 * j);
                if (d < d1) {
                    d2 = d1; second = m;
                    d1 = d; m = j;
                } else if (d == d1) {
                    double kp_j = k[0] * sites[3 * j] + k[1] * sites[3 * j + 1] + k[2] * sites[3 * j + 2];
                    double kp_m = k[0] * sites[3 * m] + k[1] * sites[3 * m + 1] + k[2] * sites[3 * m + 2];
                    d2 = d; second = j;
                    if (kp_j > kp_m) { second = m; m = j; }
                } else if (d < d2) {
                    d2 = d; second = j;
                }
            }
            start = (int32_t)m;
            if (second >= 0 && L > 0.0) {
                double g = (d2 - d1) / (2.0 * sqrt(dist2(sites + 3 * m, sites + 3 * second)));
                g /= L;
                if (g < gmin) gmin = g;
                if (g <= eta) ++near;
            }

            double s_c = s0;
            int64_t steps = 0;
            const double *pm = sites + 3 * m;
            while (L > 0.0) {
                if (steps++ > M + 8) { st = ST_STEPLIMIT; break; }
                /* candidates: the wall at L and every approached bisector plane */
                double best = L, second_best = INFINITY;
                double best_den = INFINITY;     /* the wall is preferred on ties */
                int64_t win = -1;
                for (int64_t j = 0; j < M; ++j) {
                    if (j == m) continue;
                    const double *pj = sites + 3 * j;
                    double n0 = pj[0] - pm[0], n1 = pj[1] - pm[1], n2 = pj[2] - pm[2];
                    double den = n0 * k[0] + n1 * k[1] + n2 * k[2];
                    if (!(den > 0.0)) continue;
                    double w0 = 0.5 * (pj[0] + pm[0]) - r0[0];
                    double w1 = 0.5 * (pj[1] + pm[1]) - r0[1];
                    double w2 = 0.5 * (pj[2] + pm[2]) - r0[2];
                    double sj = (n0 * w0 + n1 * w1 + n2 * w2) / den;
                    if (sj < best) {
                        second_best = best;
                        best = sj; best_den = den; win = j;
                    } else if (sj == best) {
                        second_best = sj;
                        if (win >= 0 && (den > best_den || (den == best_den && j < win))) {
                            best_den = den; win = j;
                        }
                    } else if (sj < second_best) {
                        second_best = sj;
                    }
                }
                double g = (second_best - best) / L;
                if (g < gmin) gmin = g;
                if (g <= eta) ++near;

                double len = best - s_c;
                if (len > 0.0) {
                    if (count < cap && seg_cell) {
                        seg_cell[ray * cap + count] = (int32_t)m;
                        if (seg_len) seg_len[ray * cap + count] = len;
                        if (seg_end) seg_end[ray * cap + count] = best;
                    }
                    if (rho) t += kappa * rho[m] * len;
                    ++count;
                    s_c = best;
                }
                if (win < 0) break;             /* the wall: the ray leaves the box */
                m = win;
                pm = sites + 3 * m;
            }
            if (st == ST_OK && count > cap && seg_cell) st = ST_OVERFLOW;
        }
        nseg[ray] = count;
        if (tau) tau[ray] = t;
        if (chord) chord[ray] = L;
        if (status) status[ray] = st;
        if (n_near) n_near[ray] = near;
        if (min_gap) min_gap[ray] = gmin;
        if (cell0) cell0[ray] = start;
        if (start_s) start_s[ray] = s0;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Cell faces by brute force: for cell i, every other site j and every box
 * wall is a candidate face. The candidate's plane (the bisector of p_i and
 * p_j, Eq. 3, or the wall plane) is cut to a convex polygon by the box and by
 * the half-spaces {x : |x - p_i| <= |x - p_k|} of every other site k. What is
 * left is the face of the clipped cell on that plane; j (or the wall) is a
 * face neighbour when the face has positive area. The cell volume is the sum
 * over faces of area * (distance from p_i to the face plane) / 3. The
 * cell is convex, so its bounding box is that of its vertices (Sect. 2.3),
 * the corners of its faces.
 * ------------------------------------------------------------------------- */

typedef struct { double x, y, z; } v3;

static v3 v3sub(v3 a, v3 b) { v3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static v3 v3add(v3 a, v3 b) { v3 r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static v3 v3scale(v3 a, double s) { v3 r = {a.x * s, a.y * s, a.z * s}; return r; }
static double v3dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 v3cross(v3 a, v3 b)
{
    v3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}

/* keep {x : a.x <= b}; Sutherland-Hodgman on a convex polygon */
static int clip_poly(const v3 *in, int n, v3 *out, v3 a, double b)
{
    int m = 0;
    for (int e = 0; e < n; ++e) {
        v3 P = in[e], Q = in[(e + 1) % n];
        double fp = v3dot(a, P) - b, fq = v3dot(a, Q) - b;
        if (fp <= 0.0) out[m++] = P;
        if ((fp < 0.0 && fq > 0.0) || (fp > 0.0 && fq < 0.0)) {
            double u = fp / (fp - fq);
            out[m++] = v3add(P, v3scale(v3sub(Q, P), u));
        }
    }
    return m;
}

static double poly_area(const v3 *p, int n)
{
    if (n < 3) return 0.0;
    v3 acc = {0, 0, 0};
    for (int e = 1; e + 1 < n; ++e)
        acc = v3add(acc, v3cross(v3sub(p[e], p[0]), v3sub(p[e + 1], p[0])));
    return 0.5 * sqrt(v3dot(acc, acc));
}

typedef struct { double d; int64_t j; } dj_t;
static int cmp_dj(const void *a, const void *b)
{
    const dj_t *x = (const dj_t *)a, *y = (const dj_t *)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->j < y->j) ? -1 : (x->j > y->j);
}

/* face of cell i on the plane {x : nrm.x = off}, clipped by box and all
 * sites; a face of positive area widens bb (min xyz, max xyz) to its corners */
static double face_area(const double *sites, int64_t M, const double *box, int64_t i,
                        v3 nrm, double off, int skip_wall, int64_t skip_site,
                        const dj_t *order, v3 *buf0, v3 *buf1, double *bb)
{
    double nn = sqrt(v3dot(nrm, nrm));
    v3 nh = v3scale(nrm, 1.0 / nn);
    v3 bc = {0.5 * (box[0] + box[3]), 0.5 * (box[1] + box[4]), 0.5 * (box[2] + box[5])};
    double diag = sqrt((box[3] - box[0]) * (box[3] - box[0]) + (box[4] - box[1]) * (box[4] - box[1]) +
                       (box[5] - box[2]) * (box[5] - box[2]));
    /* centre of the starting quad: box centre projected on the plane */
    v3 c = v3sub(bc, v3scale(nh, v3dot(nh, bc) - off / nn));
    v3 e = (fabs(nh.x) <= fabs(nh.y) && fabs(nh.x) <= fabs(nh.z)) ? (v3){1, 0, 0}
         : (fabs(nh.y) <= fabs(nh.z)) ? (v3){0, 1, 0} : (v3){0, 0, 1};
    v3 u = v3cross(nh, e);
    u = v3scale(u, 1.0 / sqrt(v3dot(u, u)));
    v3 w = v3cross(nh, u);
    double R = 2.0 * diag + 1.0;
    int n = 4;
    buf0[0] = v3add(c, v3add(v3scale(u, R), v3scale(w, R)));
    buf0[1] = v3add(c, v3add(v3scale(u, -R), v3scale(w, R)));
    buf0[2] = v3add(c, v3add(v3scale(u, -R), v3scale(w, -R)));
    buf0[3] = v3add(c, v3add(v3scale(u, R), v3scale(w, -R)));
    v3 *cur = buf0, *nxt = buf1;
    /* the box: x_a >= lo_a and x_a <= hi_a */
    for (int wl = 0; wl < 6 && n >= 3; ++wl) {
        if (wl == skip_wall) continue;
        int a = wl / 2;
        v3 an = {0, 0, 0};
        double b;
        if (wl % 2 == 0) { (&an.x)[a] = -1.0; b = -box[a]; }
        else { (&an.x)[a] = 1.0; b = box[a + 3]; }
        n = clip_poly(cur, n, nxt, an, b);
        v3 *t = cur; cur = nxt; nxt = t;
    }
    v3 pi = {sites[3 * i], sites[3 * i + 1], sites[3 * i + 2]};
    for (int64_t o = 0; o < M - 1 && n >= 3; ++o) {
        int64_t k = order[o].j;
        if (k == skip_site) continue;
        v3 pk = {sites[3 * k], sites[3 * k + 1], sites[3 * k + 2]};
        v3 a = v3sub(pk, pi);
        double b = v3dot(a, v3scale(v3add(pk, pi), 0.5));
        n = clip_poly(cur, n, nxt, a, b);
        v3 *t = cur; cur = nxt; nxt = t;
    }
    double ar = poly_area(cur, n);
    if (ar > 0.0) {
        for (int e = 0; e < n; ++e) {
            const double xyz[3] = {cur[e].x, cur[e].y, cur[e].z};
            for (int a = 0; a < 3; ++a) {
                if (xyz[a] < bb[a]) bb[a] = xyz[a];
                if (xyz[a] > bb[a + 3]) bb[a + 3] = xyz[a];
            }
        }
    }
    return ar;
}

/*
 * oracle_faces -- faces of the listed cells. For each cell c = cells[q]:
 * nbr[q*cap + f] holds the neighbour index (>= 0) or wall code (-1..-6) of
 * face f, area[q*cap + f] its area (> 0), nface[q] the face count and
 * volume[q] the cell volume. Faces beyond cap are counted in nface and
 * volume but not stored. If bbox != NULL, bbox[6q..6q+5] receives the
 * bounding box of the cell {xmin, ymin, zmin, xmax, ymax, zmax}: the extreme
 * coordinates of its face corners. Returns 0, or 1 on bad arguments.
 */
int oracle_faces(const double *sites, int64_t M, const double *box,
                 const int64_t *cells, int64_t ncells, int64_t cap,
                 int32_t *nbr, double *area, int32_t *nface, double *volume, double *bbox)
{
    if (M <= 0 || ncells < 0) return 1;
    int bad = 0;
#pragma omp parallel
    {
        dj_t *order = (dj_t *)malloc(sizeof(dj_t) * (size_t)(M > 1 ? M - 1 : 1));
        v3 *b0 = (v3 *)malloc(sizeof(v3) * (size_t)(M + 16));
        v3 *b1 = (v3 *)malloc(sizeof(v3) * (size_t)(M + 16));
        if (!order || !b0 || !b1) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < ncells; ++q) {
            if (!order || !b0 || !b1) continue;
            int64_t i = cells[q];
            v3 pi = {sites[3 * i], sites[3 * i + 1], sites[3 * i + 2]};
            int64_t o = 0;
            for (int64_t j = 0; j < M; ++j) {
                if (j == i) continue;
                order[o].d = dist2(sites + 3 * i, sites + 3 * j);
                order[o].j = j;
                ++o;
            }
            qsort(order, (size_t)(M - 1), sizeof(dj_t), cmp_dj);
            int32_t nf = 0;
            double vol = 0.0;
            double bb[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
            for (int64_t o2 = 0; o2 < M - 1; ++o2) {
                int64_t j = order[o2].j;
                v3 pj = {sites[3 * j], sites[3 * j + 1], sites[3 * j + 2]};
                v3 a = v3sub(pj, pi);
                double b = v3dot(a, v3scale(v3add(pj, pi), 0.5));
                double ar = face_area(sites, M, box, i, a, b, -1, j, order, b0, b1, bb);
                if (ar > 0.0) {
                    if (nf < cap) {
                        nbr[q * cap + nf] = (int32_t)j;
                        area[q * cap + nf] = ar;
                    }
                    ++nf;
                    vol += ar * (0.5 * sqrt(v3dot(a, a))) / 3.0;
                }
            }
            for (int wl = 0; wl < 6; ++wl) {
                int ax = wl / 2;
                v3 an = {0, 0, 0};
                double b;
                if (wl % 2 == 0) { (&an.x)[ax] = -1.0; b = -box[ax]; }
                else { (&an.x)[ax] = 1.0; b = box[ax + 3]; }
                double ar = face_area(sites, M, box, i, an, b, wl, -1, order, b0, b1, bb);
                if (ar > 0.0) {
                    if (nf < cap) {
                        nbr[q * cap + nf] = -(wl + 1);
                        area[q * cap + nf] = ar;
                    }
                    ++nf;
                    double h = (wl % 2 == 0) ? ((&pi.x)[ax] - box[ax]) : (box[ax + 3] - (&pi.x)[ax]);
                    vol += ar * h / 3.0;
                }
            }
            nface[q] = nf;
            volume[q] = vol;
            if (bbox)
                for (int a = 0; a < 6; ++a) bbox[6 * q + a] = bb[a];
        }
        free(order);
        free(b0);
        free(b1);
    }
    return bad;
}
