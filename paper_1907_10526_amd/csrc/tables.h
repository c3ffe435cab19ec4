// Device construction of the geometry tables (tables.hip).
#pragma once

#include "fanproj_internal.h"

namespace fanproj {

struct RayTableArgs {
    int nv, nd, beam;
    double dsd, pitch, width, pixel;
    float *f32[kRayTables];   // outputs (RayTables field order); null to skip
    double *f64[kRayTables];
};

struct TileTableArgs {
    int nx, ny, nv, nd, tiles_x, tiles_y, beam;
    double pixel, dsc, dsd, pitch, width;
    double hc_max;            // largest half effective blur anywhere
};

hipError_t launch_ray_tables(const double2 *views, const RayTableArgs &a, hipStream_t s);
// maxima[0] / [1] receive the largest cell count and window width (atomicMax;
// zero them first).
hipError_t launch_tile_table(const double2 *views, const TileTableArgs &a, int4 *out, int *maxima,
                             hipStream_t s);
// (cos g_m, sin g_m) of the arc detector's cell angles g_m = s_m / D_sd, for
// m = -kBackPad .. nd + kBackPad - 1 (entry m + kBackPad), and the rotations
// (cos, sin) of t * pitch / D_sd for t < kBackMaxUnrolled in FP32 and FP64.
hipError_t launch_arc_cells(int nd, double pitch, double dsd, double2 *cells, float2 *rot,
                            double2 *rot64, hipStream_t s);

}  // namespace fanproj
