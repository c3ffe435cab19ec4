// Device construction of the geometry tables (tables.hip).
#pragma once

#include "fanproj_internal.h"

namespace fanproj {

struct RayTableArgs {
    int nv, nd;
    double dsd, tau, pixel;
    float *f32[kRayTables];   // outputs (RayTables field order); null to skip
    double *f64[kRayTables];
};

struct TileTableArgs {
    int nx, ny, nv, nd, tiles_x, tiles_y;
    double pixel, dsc, dsd, tau;
    double hc_max;            // largest half effective blur anywhere
};

hipError_t launch_ray_tables(const double2 *views, const RayTableArgs &a, hipStream_t s);
// maxima[0] / [1] receive the largest cell count and window width (atomicMax;
// zero them first).
hipError_t launch_tile_table(const double2 *views, const TileTableArgs &a, int4 *out, int *maxima,
                             hipStream_t s);

}  // namespace fanproj
