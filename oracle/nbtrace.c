/*
 * nbtrace.c -- TEST AND BENCHMARK INFRASTRUCTURE ONLY.
 *
 * The path loop of Camps, Baes & Saftly, Sect. 2.2 (Eqs. 1-5), as the paper
 * runs it on a CPU: from the current point r in cell m, every entry of the
 * cell's neighbour list is a candidate exit -- a neighbouring site j, whose
 * bisector plane (Eq. 3) the ray meets at s = n.((p_j + p_m)/2 - r)/(n.k),
 * n = p_j - p_m (Eq. 4), considered only if n.k > 0 (the sign argument), or
 * a box wall, met at the distance of Eq. 5 -- and the path leaves the cell
 * at the smallest positive s, moving r there. It is the like-for-like
 * counterpart, in FP64 on one or several cores, of the paper's timing
 * (Table 2), and is used only to time that baseline beside the oracle; the
 * neighbour lists and start cells are inputs (any correct ones).
 *
 * Unlike the oracle (brute force over all sites from the fixed origin) this
 * loop moves a running point, so its lengths carry the rounding of each
 * move; it shares no code with the oracle or the GPU library.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 *        -fno-fast-math nbtrace.c -o libnbtrace.so -lm
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * nbtrace_paths -- the path of every ray: its segment count, optical depth
 * tau = kappa * sum(rho_m * l_m) and its no-exit events (a step with no
 * positive exit, where the loop stops; the paper reports those as rare).
 *   sites    M x 3; box {xmin, ymin, zmin, xmax, ymax, zmax}
 *   row_ptr  M + 1, col: the neighbour lists, walls -1..-6 = xmin, xmax,
 *            ymin, ymax, zmin, zmax
 *   start    N start cells (the cell holding each origin; < 0: no path)
 *   threads  OpenMP threads (<= 0: the default)
 * Returns 0, or 1 on bad arguments.
 */
int nbtrace_paths(const double *sites, int64_t M, const double *box, const int64_t *row_ptr, const int32_t *col,
                  const double *rho, double kappa, const double *origins, const double *dirs, const int32_t *start,
                  int64_t N, int threads, int32_t *nseg, double *tau, int32_t *fails)
{
    if (M <= 0 || N < 0 || !sites || !box || !row_ptr || !col || !origins || !dirs || !start || !nseg) return 1;
#ifdef _OPENMP
    const int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
#endif
    for (int64_t ray = 0; ray < N; ++ray) {
        double r[3] = {origins[3 * ray], origins[3 * ray + 1], origins[3 * ray + 2]};
        double k[3] = {dirs[3 * ray], dirs[3 * ray + 1], dirs[3 * ray + 2]};
        const double kn = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
        int32_t count = 0, fail = 0;
        double t = 0.0;
        int64_t m = start[ray];
        if (m >= 0 && kn > 0.0 && isfinite(kn)) {
            for (int a = 0; a < 3; ++a) k[a] /= kn;
            for (int64_t step = 0; step <= M + 16; ++step) {
                const double *pm = sites + 3 * m;
                double best = INFINITY;
                int32_t win = 0;
                int found = 0;
                for (int64_t e = row_ptr[m]; e < row_ptr[m + 1]; ++e) {
                    const int32_t j = col[e];
                    double s;
                    if (j >= 0) {
                        const double *pj = sites + 3 * j;
                        const double n0 = pj[0] - pm[0], n1 = pj[1] - pm[1], n2 = pj[2] - pm[2];
                        const double den = n0 * k[0] + n1 * k[1] + n2 * k[2];
                        if (!(den > 0.0)) continue;
                        s = (n0 * (0.5 * (pj[0] + pm[0]) - r[0]) + n1 * (0.5 * (pj[1] + pm[1]) - r[1]) +
                             n2 * (0.5 * (pj[2] + pm[2]) - r[2])) / den;
                    } else {
                        const int w = -j - 1, a = w / 2, hi = w % 2;
                        if (hi ? !(k[a] > 0.0) : !(k[a] < 0.0)) continue;
                        s = ((hi ? box[a + 3] : box[a]) - r[a]) / k[a];
                    }
                    if (s > 0.0 && s < best) {
                        best = s;
                        win = j;
                        found = 1;
                    }
                }
                if (!found) {
                    ++fail;
                    break;
                }
                t += kappa * (rho ? rho[m] : 0.0) * best;
                ++count;
                for (int a = 0; a < 3; ++a) r[a] += best * k[a];
                if (win < 0) break;
                m = win;
            }
        }
        nseg[ray] = count;
        if (tau) tau[ray] = t;
        if (fails) fails[ray] = fail;
    }
    return 0;
}
