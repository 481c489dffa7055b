"""MI355X-native straight paths through box-clipped 3D Voronoi grids.

The compute lives in ``libvoronoi_rt.so`` (HIP for gfx950, C ABI declared in
include/voronoi_rt.h). ``paper_1310_1854_amd.vrt`` binds it with ctypes;
torch provides device memory and streams only.
"""
