// Geometry creation: validation and the FP64 per-view / per-ray tables
// (the "fan geometry" step that precedes every projection, Sec. II-A and
// eq. (13), (16), (17)), uploaded to the device once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "fanproj_internal.h"
#include "tables.h"

namespace fanproj {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool finite_positive(double x) { return std::isfinite(x) && x > 0.0; }

// View groups of the back projection: added until about kBackGroupsPerCu
// work-groups per compute unit are in flight, at most kBackMaxGroups and with
// at least 8 views per group.
int view_groups(size_t ntiles, int n_views, int cus) {
    const long want = ((long)kBackGroupsPerCu * cus + (long)ntiles - 1) / (long)ntiles;
    long groups = std::max(1L, std::min<long>(want, kBackMaxGroups));
    while (groups > 1 && n_views / groups < 8) --groups;
    return (int)groups;
}

// Whether the scan is unchanged by a quarter turn: a square grid and views
// v + k (n_views / 4), k < 4, at the angle of view v plus k pi/2 (to 1e-13
// rad, far below what FP32 entries resolve).  The quarter-turn forms of the
// projections then evaluate each entry once for four views.
bool quarter_turn_symmetric(int nx, int ny, int n_views, const double *angles) {
    if (nx != ny || n_views % 4 != 0) return false;
    const int q = n_views / 4;
    for (int v = 0; v < n_views; ++v) {
        const double d = angles[v] - angles[v % q] - (v / q) * (0.5 * M_PI);
        if (!(std::fabs(std::remainder(d, 2.0 * M_PI)) <= 1e-13)) return false;
    }
    return true;
}

// Whether a quarter-turn symmetric scan of n_views views (n_views % 8 == 0)
// is also unchanged by the reflection across the diagonal x = y: the
// reflection takes the source at angle t to pi/2 - t and detector coordinate
// s to -s (the cells are symmetric about the detector centre), so every view
// v of the first quarter needs its partner Q - v at pi/2 - t_v (Q =
// n_views / 4; to 1e-13 rad).  The octant form of the back projection then
// evaluates each entry once for eight views.
bool octant_symmetric(int n_views, const double *angles) {
    if (n_views % 8 != 0) return false;
    const int q = n_views / 4;
    for (int v = 0; v <= q; ++v) {
        const double d = angles[v % n_views] + angles[(q - v) % n_views] - 0.5 * M_PI;
        if (!(std::fabs(std::remainder(d, 2.0 * M_PI)) <= 1e-13)) return false;
    }
    return true;
}

}  // namespace

fp_status ensure_f64_tables(fp_geometry *g) {
    std::lock_guard<std::mutex> lock(g->f64_mu);
    if (g->f64_ready) return FP_OK;
    const size_t nr = (size_t)g->nv * g->nd;
    const size_t per = align_up(nr * sizeof(double), 256);
    const size_t bytes = per * kRayTables;
    hipError_t e = pool_alloc(g->device, bytes, &g->f64_block, &g->f64_cap);
    if (e != hipSuccess) {
        g->f64_block = nullptr;
        set_error("FP64 tables: allocating " + std::to_string(bytes) + " bytes failed");
        return FP_ERR_OUT_OF_MEMORY;
    }
    char *base = static_cast<char *>(g->f64_block);
    RayTableArgs ra{};
    ra.nv = g->nv; ra.nd = g->nd; ra.beam = g->beam;
    ra.dsd = g->dsd; ra.pitch = g->pitch; ra.width = g->tau; ra.pixel = g->pixel;
    for (int k = 0; k < kRayTables; ++k) ra.f64[k] = reinterpret_cast<double *>(base + k * per);
    e = launch_ray_tables(g->dev.views, ra, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        pool_release(g->device, {{g->f64_block, g->f64_cap}}, {});
        g->f64_block = nullptr;
        return device_error("FP64 tables", e);
    }
    g->dev.r64 = RayTables<double>{ra.f64[0], per / sizeof(double)};
    g->f64_bytes = bytes;
    g->f64_ready = true;
    return FP_OK;
}
}  // namespace fanproj

using namespace fanproj;

extern "C" fp_status fp_geometry_create(int32_t nx, int32_t ny, double pixel_size,
                                        double dist_source_center,
                                        double dist_source_detector, int32_t n_views,
                                        const double *view_angles, int32_t n_det,
                                        double det_width, fp_geometry **out) {
    fp_geometry_desc d{};
    d.beam = FP_FAN_FLAT;
    d.nx = nx; d.ny = ny; d.pixel_size = pixel_size;
    d.dist_source_center = dist_source_center; d.dist_source_detector = dist_source_detector;
    d.n_views = n_views; d.view_angles = view_angles;
    d.n_det = n_det; d.det_pitch = det_width; d.det_width = det_width;
    return fp_geometry_create_desc(&d, out);
}

extern "C" fp_status fp_geometry_create_desc(const fp_geometry_desc *desc, fp_geometry **out) {
    clear_error();
    if (!out) { set_error("fp_geometry_create: out is NULL"); return FP_ERR_INVALID_ARG; }
    if (!desc) { set_error("fp_geometry_create: desc is NULL"); return FP_ERR_INVALID_ARG; }
    const int beam = desc->beam;
    const int32_t nx = desc->nx, ny = desc->ny, n_views = desc->n_views, n_det = desc->n_det;
    const double pixel_size = desc->pixel_size, det_width = desc->det_width, pitch = desc->det_pitch;
    const double *view_angles = desc->view_angles;
    const bool fan = beam != FP_PARALLEL;
    // parallel beams have no source: the distances are not read
    const double dist_source_center = fan ? desc->dist_source_center : 0.0;
    const double dist_source_detector = fan ? desc->dist_source_detector : 0.0;
    if (beam != FP_FAN_FLAT && beam != FP_FAN_ARC && beam != FP_PARALLEL) {
        set_error("fp_geometry_create: unknown beam " + std::to_string(beam));
        return FP_ERR_INVALID_ARG;
    }
    if (!view_angles) { set_error("fp_geometry_create: view_angles is NULL"); return FP_ERR_INVALID_ARG; }
    if (nx < 1 || ny < 1 || n_views < 1 || n_det < 1) {
        set_error("fp_geometry_create: nx, ny, n_views and n_det must be >= 1");
        return FP_ERR_INVALID_ARG;
    }
    if (!finite_positive(pixel_size) || !finite_positive(det_width) || !finite_positive(pitch)) {
        set_error("fp_geometry_create: pixel_size, det_width and the pitch must be finite and > 0");
        return FP_ERR_INVALID_ARG;
    }
    const double half_diag = pixel_size * 0.5 * std::sqrt((double)nx * nx + (double)ny * ny);
    if (fan) {
        if (!finite_positive(dist_source_center) || !std::isfinite(dist_source_detector)) {
            set_error("fp_geometry_create: the distances must be finite and > 0");
            return FP_ERR_INVALID_ARG;
        }
        if (!(dist_source_detector > dist_source_center)) {
            set_error("fp_geometry_create: dist_source_detector must exceed dist_source_center");
            return FP_ERR_INVALID_ARG;
        }
        if (!(dist_source_center > half_diag + pixel_size)) {
            set_error("fp_geometry_create: the source must lie outside the image "
                      "(dist_source_center > pixel_size * (sqrt(nx^2+ny^2)/2 + 1))");
            return FP_ERR_INVALID_ARG;
        }
    }
    if (beam == FP_FAN_ARC &&
        !(0.5 * n_det * pitch + 0.5 * det_width < 80.0 * M_PI / 180.0 * dist_source_detector)) {
        set_error("fp_geometry_create: the arc detector must stay within 80 degrees of the "
                  "central ray ((n_det/2) * det_pitch + det_width/2 < 1.396 * dist_source_detector)");
        return FP_ERR_INVALID_ARG;
    }
    for (int v = 0; v < n_views; ++v)
        if (!std::isfinite(view_angles[v])) {
            set_error("fp_geometry_create: view angle " + std::to_string(v) + " is not finite");
            return FP_ERR_INVALID_ARG;
        }
    if ((int64_t)n_views * n_det > (int64_t)1 << 30 || (int64_t)nx * ny > (int64_t)1 << 30) {
        set_error("fp_geometry_create: problem too large for 32-bit ray / pixel indices");
        return FP_ERR_UNSUPPORTED;
    }

    auto g = std::make_unique<fp_geometry>();
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return device_error("hipGetDevice", e);
    g->nx = nx; g->ny = ny; g->nv = n_views; g->nd = n_det; g->beam = beam;
    g->pixel = pixel_size; g->dsc = dist_source_center; g->dsd = dist_source_detector;
    g->tau = det_width;
    g->pitch = pitch;
    g->angles.assign(view_angles, view_angles + n_views);

    const size_t nr = (size_t)n_views * n_det;
    const int tiles_x = (nx + kBackTileW - 1) / kBackTileW;
    const int tiles_y = (ny + kBackTileH - 1) / kBackTileH;
    const size_t ntiles = (size_t)tiles_x * tiles_y;

    // ---- per-view table on the host; everything per ray / per tile on the device ----
    std::vector<double> views(2 * (size_t)n_views);
    for (int v = 0; v < n_views; ++v) {
        views[2 * v] = std::cos(view_angles[v]);
        views[2 * v + 1] = std::sin(view_angles[v]);
    }
    const double D = dist_source_detector, tau = det_width, delta = pixel_size;
    const double c0 = 0.5 * (n_det - 1);
    // Largest half effective blur anywhere: tau'/2 = g L / 2 with
    // L <= D_sc + (radius of the image) (fan), or tau / 2 (parallel).
    double hc_max = 0.5 * tau;
    if (beam == FP_FAN_FLAT) {
        double gmax = 0.0;
        for (int m = 0; m < n_det; ++m) {
            const double s = (m - c0) * pitch;
            gmax = std::max(gmax, 0.5 * tau * D *
                                      (1.0 / (D * D + s * (s + 0.5 * tau)) +
                                       1.0 / (D * D + s * (s - 0.5 * tau))));
        }
        hc_max = 0.5 * gmax * (dist_source_center + half_diag + delta);
    } else if (beam == FP_FAN_ARC) {
        hc_max = std::tan(0.5 * tau / D) * (dist_source_center + half_diag + delta);
    }

    // ---- device block: views, per-ray tables, per-tile table, arc cells, two maxima ----
    const size_t A = 256;
    const size_t n_arc = beam == FP_FAN_ARC ? (size_t)n_det + 2 * kBackPad : 0;
    size_t off = 0;
    const size_t off_views = off; off = align_up(off + views.size() * sizeof(double), A);
    // the per-ray tables, equally spaced (RayTables)
    const size_t ray_per = align_up(nr * sizeof(float), A);
    const size_t off_rays = off; off += kRayTables * ray_per;
    const size_t off_tiles = off; off = align_up(off + (size_t)n_views * ntiles * sizeof(int4), A);
    const size_t off_arc = off; off = align_up(off + n_arc * sizeof(double2), A);
    const size_t off_rot = off; off = align_up(off + (n_arc ? kBackMaxUnrolled : 0) * sizeof(float2), A);
    const size_t off_rot64 = off; off = align_up(off + (n_arc ? kBackMaxUnrolled : 0) * sizeof(double2), A);
    const size_t off_max = off; off = align_up(off + 2 * sizeof(int), A);
    g->table_bytes = off;
    e = pool_alloc(g->device, g->table_bytes, &g->table_block, &g->table_cap);
    if (e != hipSuccess) {
        g->table_block = nullptr;
        set_error("fp_geometry_create: allocating " + std::to_string(g->table_bytes) +
                  " bytes failed: " + hipGetErrorString(e));
        return FP_ERR_OUT_OF_MEMORY;
    }
    char *base = static_cast<char *>(g->table_block);
    auto fail = [&](const char *what, hipError_t err) {
        (void)hipDeviceSynchronize();   // (the tables' own kernels may be queued)
        (void)hipGetLastError();
        pool_release(g->device, {{g->table_block, g->table_cap}}, {});
        g->table_block = nullptr;
        return device_error(what, err);
    };
    e = hipMemcpy(base + off_views, views.data(), views.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail("fp_geometry_create: view table upload", e);
    e = hipMemset(base + off_max, 0, 2 * sizeof(int));
    if (e != hipSuccess) return fail("fp_geometry_create: hipMemset", e);
    const double2 *d_views = reinterpret_cast<const double2 *>(base + off_views);
    RayTableArgs ra{};
    ra.nv = n_views; ra.nd = n_det; ra.beam = beam;
    ra.dsd = D; ra.pitch = pitch; ra.width = tau; ra.pixel = delta;
    for (int k = 0; k < kRayTables; ++k)
        ra.f32[k] = reinterpret_cast<float *>(base + off_rays + k * ray_per);
    e = launch_ray_tables(d_views, ra, nullptr);
    if (e != hipSuccess) return fail("fp_geometry_create: ray tables", e);
    TileTableArgs ta{};
    ta.nx = nx; ta.ny = ny; ta.nv = n_views; ta.nd = n_det; ta.tiles_x = tiles_x; ta.tiles_y = tiles_y;
    ta.beam = beam;
    ta.pixel = delta; ta.dsc = dist_source_center; ta.dsd = D; ta.pitch = pitch; ta.width = tau;
    ta.hc_max = hc_max;
    int4 *d_tiles = reinterpret_cast<int4 *>(base + off_tiles);
    int *d_max = reinterpret_cast<int *>(base + off_max);
    e = launch_tile_table(d_views, ta, d_tiles, d_max, nullptr);
    if (e != hipSuccess) return fail("fp_geometry_create: tile table", e);
    double2 *d_arc = n_arc ? reinterpret_cast<double2 *>(base + off_arc) : nullptr;
    float2 *d_rot = n_arc ? reinterpret_cast<float2 *>(base + off_rot) : nullptr;
    double2 *d_rot64 = n_arc ? reinterpret_cast<double2 *>(base + off_rot64) : nullptr;
    if (d_arc) {
        e = launch_arc_cells(n_det, pitch, D, d_arc, d_rot, d_rot64, nullptr);
        if (e != hipSuccess) return fail("fp_geometry_create: arc cells", e);
    }
    int maxima[2] = {0, 0};
    e = hipMemcpy(maxima, d_max, sizeof(maxima), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail("fp_geometry_create: tables", e);
    const int max_cells = maxima[0];

    DevGeom &d = g->dev;
    d.nx = nx; d.ny = ny; d.nv = n_views; d.nd = n_det;
    d.tiles_x = tiles_x; d.tiles_y = tiles_y;
    d.max_cells = max_cells;
    d.beam = beam;
    d.pixel = delta; d.dsc = dist_source_center; d.dsd = D; d.tau = tau; d.pitch = pitch;
    d.cell_step = beam == FP_FAN_ARC ? pitch / D : pitch;
    d.half_diag = half_diag + delta;
    d.views = d_views;
    d.arc_cells = d_arc;
    d.arc_rot = d_rot;
    d.arc_rot64 = d_rot64;
    d.r32 = RayTables<float>{ra.f32[0], ray_per / sizeof(float)};
    d.r64 = RayTables<double>{};
    d.tile_cells = d_tiles;
    // The walk's window spans the support |s'| < hab + hc along the cross
    // axis, where s' advances by at least kFwdCrossMin delta per pixel and
    // hab <= delta / sqrt(2): at most floor(2 hq) + 1 pixels with
    // hq = (0.7072 delta + hc_max) / (kFwdCrossMin delta).
    d.fwd_window =
        (int)std::floor(2.0 * (0.7072 * delta + hc_max) / (kFwdCrossMin * delta)) + 1;
    d.back_cap = 0;
    for (int cap : kBackCaps)
        if (max_cells + 2 * kBackPad <= cap) { d.back_cap = cap; break; }
    if (d.back_cap == 0 || back_max_batch<float>(d) < 1) {
        pool_release(g->device, {{g->table_block, g->table_cap}}, {});
        g->table_block = nullptr;
        set_error("fp_geometry_create: a back-projection tile spans " + std::to_string(max_cells) +
                  " cells, more than the on-chip staging holds (" + std::to_string(kBackMaxCap) +
                  "; cells too narrow for the pixel size)");
        return FP_ERR_UNSUPPORTED;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess ||
        cus < 1) {
        (void)hipGetLastError();
        cus = 256;
    }
    d.back_groups = view_groups(ntiles, n_views, cus);
    g->quarter = quarter_turn_symmetric(nx, ny, n_views, view_angles) &&
                 back_max_batch<float>(d) >= 4;
    if (g->quarter) {
        g->dev_quarter = d;
        g->dev_quarter.nv = n_views / 4;
        g->dev_quarter.back_groups = view_groups(ntiles, n_views / 4, cus);
    }
    g->octant = g->quarter && octant_symmetric(n_views, view_angles) &&
                back_max_batch<float>(d) >= 8;
    if (g->octant) {
        g->dev_octant = d;
        g->dev_octant.nv = n_views / 8 + 1;
        g->dev_octant.quarter_views = n_views / 4;
        g->dev_octant.back_groups = view_groups(ntiles, n_views / 8 + 1, cus);
    }
    *out = g.release();
    return FP_OK;
}

extern "C" fp_status fp_geometry_destroy(fp_geometry *g) {
    clear_error();
    if (!g) return FP_OK;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != g->device) e = hipSetDevice(g->device);
    if (e == hipSuccess) {
        // The blocks go back to the pool with the marks of the work queued
        // with the geometry (the latest launches on every stream that used
        // it); nothing waits here.  Without a complete record of that work,
        // wait for the device instead.
        std::vector<MarkPtr> after;
        {
            std::lock_guard<std::mutex> lock(g->use_mu);
            for (auto &u : g->uses) after.push_back(u.second);
            g->uses.clear();
            if (g->untracked) e = hipDeviceSynchronize();
        }
        pool_release(g->device,
                     {{g->table_block, g->table_cap}, {g->f64_block, g->f64_cap},
                      {g->row_w, g->row_cap}, {g->col_w, g->col_cap}},
                     after);
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    delete g;
    if (e != hipSuccess) return device_error("fp_geometry_destroy", e);
    return FP_OK;
}

extern "C" size_t fp_geometry_device_bytes(const fp_geometry *g) {
    if (!g) return 0;
    return g->table_bytes + g->f64_bytes + g->weight_bytes;
}

extern "C" int32_t fp_geometry_quarter_turn(const fp_geometry *g) { return g && g->quarter ? 1 : 0; }

extern "C" int32_t fp_geometry_symmetry(const fp_geometry *g) {
    if (!g) return 0;
    return g->octant ? 8 : g->quarter ? 4 : 1;
}
