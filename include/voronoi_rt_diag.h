/*
 * voronoi_rt_diag.h -- diagnostic entry points of libvoronoi_rt. They break
 * a grid on purpose, to test how the library recovers; they are not for
 * use on grids whose paths matter. The rest of the ABI is voronoi_rt.h.
 */
#ifndef VORONOI_RT_DIAG_H
#define VORONOI_RT_DIAG_H

#include "voronoi_rt.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * vor_grid_truncate_row -- keeps only the first `keep` entries (internal
 * order) of the neighbour list of site `site` (user index), so that the
 * table misses faces of that cell and paths through it take the no-exit
 * fallback of Sect. 2.2 (advance a small distance, locate the point again).
 * Paths are no longer exact after this; it exists to test that recovery.
 * Synchronous; VOR_EINVAL for a bad site or a negative keep.
 */
vor_status vor_grid_truncate_row(vor_grid *grid, int64_t site, int32_t keep);

#ifdef __cplusplus
}
#endif
#endif /* VORONOI_RT_DIAG_H */
