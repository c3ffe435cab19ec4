// Geometry creation: validation and the FP64 per-view / per-ray tables
// (the "fan geometry" step that precedes every projection, Sec. II-A and
// eq. (13), (16), (17)), uploaded to the device once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "fanproj_internal.h"

namespace fanproj {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool finite_positive(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

void compute_ray_constants(const fp_geometry &g, std::vector<double> (&out)[kRayTables]) {
    const size_t nr = (size_t)g.nv * g.nd;
    for (auto &v : out) v.assign(nr, 0.0);
    const double D = g.dsd, tau = g.tau, delta = g.pixel, c0 = 0.5 * (g.nd - 1);
    for (int v = 0; v < g.nv; ++v) {
        const double cs = std::cos(g.angles[v]), sn = std::sin(g.angles[v]);
        // u = (cs, sn) towards the source; e = (sn, -cs) along the detector.
        for (int m = 0; m < g.nd; ++m) {
            const double s = (m - c0) * tau;
            const double R = std::sqrt(D * D + s * s);
            // w_perp = (D e + s u) / R: unit normal of the ray through s.
            const double wpx = (D * sn + s * cs) / R;
            const double wpy = (-D * cs + s * sn) / R;
            const double z1 = delta * std::fabs(wpx), z2 = delta * std::fabs(wpy);
            const double a = std::min(z1, z2), b = std::max(z1, z2);
            // eq. (17): tau' = L * (tan_hi - tan_lo) with
            // tan_(+-) = D (s_(+-) - s) / (D^2 + s s_(+-)), s_(+-) = s +- tau/2.
            const double gm = 0.5 * tau * D *
                              (1.0 / (D * D + s * (s + 0.5 * tau)) +
                               1.0 / (D * D + s * (s - 0.5 * tau)));
            const double a_safe = std::max(a, 1e-30);
            const size_t r = (size_t)v * g.nd + m;
            out[0][r] = 1.0 / R;                        // inv_r
            out[1][r] = gm / (2.0 * R);                 // ghr
            out[2][r] = 0.5 * (a + b);                  // hab
            out[3][r] = 1.0 / a_safe;                   // ia
            out[4][r] = -0.5 * (b - a) / a_safe;        // nhbia
            out[5][r] = 0.5 * a;                        // ha
            out[6][r] = delta * delta / (2.0 * b);      // wb
        }
    }
}

fp_status ensure_f64_tables(fp_geometry *g) {
    std::lock_guard<std::mutex> lock(g->f64_mu);
    if (g->f64_ready) return FP_OK;
    const size_t nr = (size_t)g->nv * g->nd;
    std::vector<double> rays64[kRayTables];
    compute_ray_constants(*g, rays64);
    const size_t per = align_up(nr * sizeof(double), 256);
    const size_t bytes = per * kRayTables;
    hipError_t e = hipMalloc(&g->f64_block, bytes);
    if (e != hipSuccess) {
        g->f64_block = nullptr;
        (void)hipGetLastError();
        set_error("FP64 tables: hipMalloc of " + std::to_string(bytes) + " bytes failed");
        return FP_ERR_OUT_OF_MEMORY;
    }
    std::vector<char> host(bytes, 0);
    for (int k = 0; k < kRayTables; ++k)
        std::memcpy(host.data() + k * per, rays64[k].data(), nr * sizeof(double));
    e = hipMemcpy(g->f64_block, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(g->f64_block);
        g->f64_block = nullptr;
        return device_error("FP64 tables: upload", e);
    }
    const char *base = static_cast<const char *>(g->f64_block);
    const double *t[kRayTables];
    for (int k = 0; k < kRayTables; ++k) t[k] = reinterpret_cast<const double *>(base + k * per);
    g->dev.r64 = RayTables<double>{t[0], t[1], t[2], t[3], t[4], t[5], t[6]};
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
    clear_error();
    if (!out) { set_error("fp_geometry_create: out is NULL"); return FP_ERR_INVALID_ARG; }
    if (!view_angles) { set_error("fp_geometry_create: view_angles is NULL"); return FP_ERR_INVALID_ARG; }
    if (nx < 1 || ny < 1 || n_views < 1 || n_det < 1) {
        set_error("fp_geometry_create: nx, ny, n_views and n_det must be >= 1");
        return FP_ERR_INVALID_ARG;
    }
    if (!finite_positive(pixel_size) || !finite_positive(det_width) ||
        !finite_positive(dist_source_center) || !std::isfinite(dist_source_detector)) {
        set_error("fp_geometry_create: pixel_size, det_width and the distances must be finite and > 0");
        return FP_ERR_INVALID_ARG;
    }
    if (!(dist_source_detector > dist_source_center)) {
        set_error("fp_geometry_create: dist_source_detector must exceed dist_source_center");
        return FP_ERR_INVALID_ARG;
    }
    const double half_diag = pixel_size * 0.5 * std::sqrt((double)nx * nx + (double)ny * ny);
    if (!(dist_source_center > half_diag + pixel_size)) {
        set_error("fp_geometry_create: the source must lie outside the image "
                  "(dist_source_center > pixel_size * (sqrt(nx^2+ny^2)/2 + 1))");
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
    g->nx = nx; g->ny = ny; g->nv = n_views; g->nd = n_det;
    g->pixel = pixel_size; g->dsc = dist_source_center; g->dsd = dist_source_detector;
    g->tau = det_width;
    g->angles.assign(view_angles, view_angles + n_views);

    const size_t nr = (size_t)n_views * n_det;
    const int tiles_x = (nx + kBackTileW - 1) / kBackTileW;
    const int tiles_y = (ny + kBackTileH - 1) / kBackTileH;
    const size_t ntiles = (size_t)tiles_x * tiles_y;

    // ---- host tables (FP64 arithmetic) ----
    std::vector<double> views(2 * (size_t)n_views);
    std::vector<int32_t> tile_cells(4 * (size_t)n_views * ntiles);
    const double D = dist_source_detector, tau = det_width, delta = pixel_size;
    const double c0 = 0.5 * (n_det - 1);
    int max_cells = 0;
    for (int v = 0; v < n_views; ++v) {
        views[2 * v] = std::cos(view_angles[v]);
        views[2 * v + 1] = std::sin(view_angles[v]);
    }
    std::vector<double> rays64[kRayTables];
    compute_ray_constants(*g, rays64);
    // Largest half effective blur anywhere: tau'/2 = g_m L / 2 with
    // L <= D_sc D / R_m + (radius of the image) <= D_sc + half_diag + delta.
    double gmax = 0.0;
    for (int m = 0; m < n_det; ++m) {
        const double s = (m - c0) * tau;
        gmax = std::max(gmax, 0.5 * tau * D *
                                  (1.0 / (D * D + s * (s + 0.5 * tau)) +
                                   1.0 / (D * D + s * (s - 0.5 * tau))));
    }
    const double hc_max = 0.5 * gmax * (dist_source_center + half_diag + delta);
    // Cells that any pixel of a back-projection tile can touch.  A non-zero
    // entry needs the ray through the cell centre to pass within hab + hc of
    // the pixel centre, i.e. to cross the pixel dilated by hc <= hc_max; so
    // the ray crosses the tile rectangle dilated by hc_max, whose detector
    // shadow is spanned by its corners.  One guard cell on each side.
    //
    // Window of one pixel k: its non-zero cells satisfy |s_m - s_k| < H_k
    // with s_k = D (e.k) / h_k its centre's shadow.  From s' = h (s_k - s_m) / R_m
    // and the support |s'| < hab + hc: the pixel term hab R / h equals
    // delta P(s_m) / (2h) with P(s) = |D sin + s cos| + |-D cos + s sin|
    // (Lipschitz constant sqrt 2); the blur term hc R / h is at most
    // kappa tau/2 (1 + |s_m - s_k| / (2D)), kappa = 1 / (1 - tau^2 / (16 D^2)).
    // Solved for |s_m - s_k|:
    //   H_k = (delta P(s_k) / (2 h_k) + kappa tau / 2) / (1 - delta / (sqrt2 h_k) - kappa tau / (4D)).
    // Over a tile P(s_k) is largest at an end of the tile's shadow (P is
    // convex) and h_k smallest at a corner, which bounds H_k by H_tile; the
    // window of every pixel of the tile then holds T = floor(2 H / tau) + 1 cells.
    const double kappa = 1.0 / (1.0 - tau * tau / (16.0 * D * D));
    const double x0 = -0.5 * (nx - 1) * delta, y0 = -0.5 * (ny - 1) * delta;
    int max_window = 0;
    for (int v = 0; v < n_views; ++v) {
        const double cs = views[2 * v], sn = views[2 * v + 1];
        auto P = [&](double s) { return std::fabs(D * sn + s * cs) + std::fabs(-D * cs + s * sn); };
        for (int ty = 0; ty < tiles_y; ++ty)
            for (int tx = 0; tx < tiles_x; ++tx) {
                const int i0 = tx * kBackTileW, i1 = std::min(nx, i0 + kBackTileW) - 1;
                const int j0 = ty * kBackTileH, j1 = std::min(ny, j0 + kBackTileH) - 1;
                const double ex[2] = {x0 + (i0 - 0.5) * delta, x0 + (i1 + 0.5) * delta};
                const double ey[2] = {y0 + (j0 - 0.5) * delta, y0 + (j1 + 0.5) * delta};
                double smin = INFINITY, smax = -INFINITY, hmin = INFINITY;
                double dmin = INFINITY, dmax = -INFINITY;
                bool in_front = true;
                for (int cx = 0; cx < 2; ++cx)
                    for (int cy = 0; cy < 2; ++cy) {
                        const double x = ex[cx], y = ey[cy];
                        const double depth = dist_source_center - (cs * x + sn * y);
                        const double sh = D * (sn * x - cs * y) / depth;
                        smin = std::min(smin, sh);
                        smax = std::max(smax, sh);
                        hmin = std::min(hmin, depth);
                        // dilated corner
                        const double xd = x + (cx ? hc_max : -hc_max), yd = y + (cy ? hc_max : -hc_max);
                        const double dd = dist_source_center - (cs * xd + sn * yd);
                        if (!(dd > 0.0)) in_front = false;
                        const double shd = D * (sn * xd - cs * yd) / dd;
                        dmin = std::min(dmin, shd);
                        dmax = std::max(dmax, shd);
                    }
                long lo = 0, hi = n_det - 1;
                if (in_front) {
                    lo = std::max((long)std::ceil(dmin / tau + c0) - 1, 0L);
                    hi = std::min((long)std::floor(dmax / tau + c0) + 1, (long)n_det - 1);
                }
                const int cnt = hi >= lo ? (int)(hi - lo + 1) : 0;
                const double den = 1.0 - delta / (std::sqrt(2.0) * hmin) - kappa * tau / (4.0 * D);
                double H = (delta * std::max(P(smin), P(smax)) / (2.0 * hmin) + 0.5 * kappa * tau) / den;
                // margin for the FP32 shadow and window start computed per pixel
                H = H * (1.0 + 1e-5) + 1e-3 * tau + 1e-6 * std::max(std::fabs(smin), std::fabs(smax));
                // (capped far above any staged range; the kernel clamps a window
                // to the staged cells, which hold every non-zero cell)
                const double Td = std::floor(2.0 * H / tau) + 1.0;
                int T = den > 0.0 && Td < (double)(1 << 20) ? (int)Td : (1 << 20);
                const float Hf = (float)H;
                int32_t Hbits;
                std::memcpy(&Hbits, &Hf, sizeof(Hbits));
                const size_t t = ((size_t)v * ntiles + (size_t)ty * tiles_x + tx) * 4;
                tile_cells[t] = cnt ? (int32_t)lo : 0;
                tile_cells[t + 1] = cnt;
                tile_cells[t + 2] = T;
                tile_cells[t + 3] = Hbits;
                max_cells = std::max(max_cells, cnt);
                max_window = std::max(max_window, T);
            }
    }

    // ---- device block ----
    const size_t A = 256;
    size_t off = 0;
    const size_t off_views = off; off = align_up(off + views.size() * sizeof(double), A);
    size_t off_rays[kRayTables];
    for (int k = 0; k < kRayTables; ++k) { off_rays[k] = off; off = align_up(off + nr * sizeof(float), A); }
    const size_t off_tiles = off; off = align_up(off + tile_cells.size() * sizeof(int32_t), A);
    g->table_bytes = off;

    DevGeom &d = g->dev;
    d.nx = nx; d.ny = ny; d.nv = n_views; d.nd = n_det;
    d.tiles_x = tiles_x; d.tiles_y = tiles_y;
    d.max_cells = max_cells;
    d.pixel = delta; d.dsc = dist_source_center; d.dsd = D; d.tau = tau;
    d.half_diag = half_diag + delta;
    d.back_cap = 0;
    (void)max_window;
    for (int cap : kBackCaps)
        if (max_cells + 2 * kBackPad <= cap) { d.back_cap = cap; break; }
    if (d.back_cap == 0) {
        set_error("fp_geometry_create: a back-projection tile spans " + std::to_string(max_cells) +
                  " cells, more than the on-chip staging holds (" + std::to_string(kBackMaxCap) +
                  "; cells too narrow for the pixel size)");
        return FP_ERR_UNSUPPORTED;
    }
    if (back_max_batch<float>(d) < 1) {
        set_error("fp_geometry_create: a back-projection tile spans " + std::to_string(max_cells) +
                  " cells, more than the on-chip staging holds");
        return FP_ERR_UNSUPPORTED;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess ||
        cus < 1) {
        (void)hipGetLastError();
        cus = 256;
    }
    {
        const long want = ((long)kBackGroupsPerCu * cus + (long)ntiles - 1) / (long)ntiles;
        long groups = std::max(1L, std::min<long>(want, kBackMaxGroups));
        while (groups > 1 && n_views / groups < 8) --groups;
        d.back_groups = (int)groups;
    }
    e = hipMalloc(&g->table_block, g->table_bytes);
    if (e != hipSuccess) {
        g->table_block = nullptr;
        (void)hipGetLastError();
        set_error("fp_geometry_create: hipMalloc of " + std::to_string(g->table_bytes) +
                  " bytes failed: " + hipGetErrorString(e));
        return FP_ERR_OUT_OF_MEMORY;
    }
    char *base = static_cast<char *>(g->table_block);
    std::vector<char> host(g->table_bytes, 0);
    std::memcpy(host.data() + off_views, views.data(), views.size() * sizeof(double));
    for (int k = 0; k < kRayTables; ++k) {
        float *dst = reinterpret_cast<float *>(host.data() + off_rays[k]);
        for (size_t r = 0; r < nr; ++r) dst[r] = (float)rays64[k][r];
    }
    std::memcpy(host.data() + off_tiles, tile_cells.data(), tile_cells.size() * sizeof(int32_t));
    e = hipMemcpy(base, host.data(), g->table_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(g->table_block);
        return device_error("fp_geometry_create: table upload", e);
    }
    d.views = reinterpret_cast<const double2 *>(base + off_views);
    const float *fr[kRayTables];
    for (int k = 0; k < kRayTables; ++k) fr[k] = reinterpret_cast<const float *>(base + off_rays[k]);
    d.r32 = RayTables<float>{fr[0], fr[1], fr[2], fr[3], fr[4], fr[5], fr[6]};
    d.r64 = RayTables<double>{};
    d.tile_cells = reinterpret_cast<const int4 *>(base + off_tiles);
    *out = g.release();
    return FP_OK;
}

extern "C" fp_status fp_geometry_destroy(fp_geometry *g) {
    clear_error();
    if (!g) return FP_OK;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != g->device) e = hipSetDevice(g->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    hipError_t f = hipSuccess;
    if (g->table_block) f = hipFree(g->table_block);
    if (g->f64_block) (void)hipFree(g->f64_block);
    if (g->row_w) (void)hipFree(g->row_w);
    if (g->col_w) (void)hipFree(g->col_w);
    if (cur != g->device) (void)hipSetDevice(cur);
    delete g;
    if (e != hipSuccess) return device_error("fp_geometry_destroy", e);
    if (f != hipSuccess) return device_error("fp_geometry_destroy: hipFree", f);
    return FP_OK;
}

extern "C" size_t fp_geometry_device_bytes(const fp_geometry *g) {
    if (!g) return 0;
    return g->table_bytes + g->f64_bytes + g->weight_bytes;
}
