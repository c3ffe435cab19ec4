// Geometry tables built on the device (FP64 arithmetic): the per-ray
// constants of eq. (13), (16), (17) and the per-(view, tile) cell ranges and
// window bounds of the back projection.  One thread per ray and one per
// (view, tile); the host supplies only the per-view cosines and sines.
#include "fanproj_internal.h"
#include "tables.h"

namespace fanproj {
namespace {

__global__ __launch_bounds__(256) void ray_tables_kernel(const double2 *__restrict__ views,
                                                         RayTableArgs a) {
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (size_t)a.nv * a.nd) return;
    const int v = (int)(r / a.nd), m = (int)(r % a.nd);
    const double cs = views[v].x, sn = views[v].y;
    const double D = a.dsd, tau = a.tau, delta = a.pixel;
    // u = (cs, sn) towards the source; e = (sn, -cs) along the detector.
    const double s = (m - 0.5 * (a.nd - 1)) * tau;
    const double R = sqrt(D * D + s * s);
    // w_perp = (D e + s u) / R: unit normal of the ray through s.
    const double wpx = (D * sn + s * cs) / R;
    const double wpy = (-D * cs + s * sn) / R;
    const double z1 = delta * fabs(wpx), z2 = delta * fabs(wpy);
    const double lo = fmin(z1, z2), hi = fmax(z1, z2);
    // eq. (17): tau' = L * (tan_hi - tan_lo) with
    // tan_(+-) = D (s_(+-) - s) / (D^2 + s s_(+-)), s_(+-) = s +- tau/2.
    const double gm = 0.5 * tau * D * (1.0 / (D * D + s * (s + 0.5 * tau)) +
                                       1.0 / (D * D + s * (s - 0.5 * tau)));
    const double a_safe = fmax(lo, 1e-30);
    const double val[kRayTables] = {
        1.0 / R,                       // inv_r
        gm / (2.0 * R),                // ghr
        0.5 * (lo + hi),               // hab
        1.0 / a_safe,                  // ia
        -0.5 * (hi - lo) / a_safe,     // nhbia
        0.5 * lo,                      // ha
        delta * delta / (2.0 * hi),    // wb
    };
#pragma unroll
    for (int k = 0; k < kRayTables; ++k) {
        if (a.f32[k]) a.f32[k][r] = (float)val[k];
        if (a.f64[k]) a.f64[k][r] = val[k];
    }
}

// Cells that any pixel of a back-projection tile can touch.  A non-zero
// entry needs the ray through the cell centre to pass within hab + hc of the
// pixel centre, i.e. to cross the pixel dilated by hc <= hc_max; so the ray
// crosses the tile rectangle dilated by hc_max, whose detector shadow is
// spanned by its corners.  One guard cell on each side.
//
// Window of one pixel k: its non-zero cells satisfy |s_m - s_k| < H_k with
// s_k = D (e.k) / h_k its centre's shadow.  From s' = h (s_k - s_m) / R_m and
// the support |s'| < hab + hc: the pixel term hab R / h equals
// delta P(s_m) / (2h) with P(s) = |D sin + s cos| + |-D cos + s sin|
// (Lipschitz constant sqrt 2); the blur term hc R / h is at most
// kappa tau/2 (1 + |s_m - s_k| / (2D)), kappa = 1 / (1 - tau^2 / (16 D^2)).
// Solved for |s_m - s_k|:
//   H_k = (delta P(s_k) / (2 h_k) + kappa tau / 2) / (1 - delta / (sqrt2 h_k) - kappa tau / (4D)).
// Over a tile P(s_k) is largest at an end of the tile's shadow (P is convex)
// and h_k smallest at a corner, which bounds H_k by H_tile; the window of
// every pixel of the tile then holds T = floor(2 H / tau) + 1 cells.
__global__ __launch_bounds__(256) void tile_table_kernel(const double2 *__restrict__ views,
                                                         TileTableArgs a,
                                                         int4 *__restrict__ out,
                                                         int *__restrict__ maxima) {
    const int ntiles = a.tiles_x * a.tiles_y;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)a.nv * ntiles) return;
    const int v = (int)(t / ntiles), tile = (int)(t % ntiles);
    const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
    const double cs = views[v].x, sn = views[v].y;
    const double D = a.dsd, tau = a.tau, delta = a.pixel, c0 = 0.5 * (a.nd - 1);
    const double x0 = -0.5 * (a.nx - 1) * delta, y0 = -0.5 * (a.ny - 1) * delta;
    const int i0 = tx * kBackTileW, i1 = min(a.nx, i0 + kBackTileW) - 1;
    const int j0 = ty * kBackTileH, j1 = min(a.ny, j0 + kBackTileH) - 1;
    const double ex[2] = {x0 + (i0 - 0.5) * delta, x0 + (i1 + 0.5) * delta};
    const double ey[2] = {y0 + (j0 - 0.5) * delta, y0 + (j1 + 0.5) * delta};
    double smin = INFINITY, smax = -INFINITY, hmin = INFINITY;
    double dmin = INFINITY, dmax = -INFINITY;
    bool in_front = true;
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy) {
            const double x = ex[cx], y = ey[cy];
            const double depth = a.dsc - (cs * x + sn * y);
            const double sh = D * (sn * x - cs * y) / depth;
            smin = fmin(smin, sh);
            smax = fmax(smax, sh);
            hmin = fmin(hmin, depth);
            const double xd = x + (cx ? a.hc_max : -a.hc_max), yd = y + (cy ? a.hc_max : -a.hc_max);
            const double dd = a.dsc - (cs * xd + sn * yd);
            if (!(dd > 0.0)) in_front = false;
            const double shd = D * (sn * xd - cs * yd) / dd;
            dmin = fmin(dmin, shd);
            dmax = fmax(dmax, shd);
        }
    long lo = 0, hi = a.nd - 1;
    if (in_front) {
        lo = max((long)ceil(dmin / tau + c0) - 1, 0L);
        hi = min((long)floor(dmax / tau + c0) + 1, (long)a.nd - 1);
    }
    const int cnt = hi >= lo ? (int)(hi - lo + 1) : 0;
    const double kappa = 1.0 / (1.0 - tau * tau / (16.0 * D * D));
    const double den = 1.0 - delta / (sqrt(2.0) * hmin) - kappa * tau / (4.0 * D);
    const double Pmax = fmax(fabs(D * sn + smin * cs) + fabs(-D * cs + smin * sn),
                             fabs(D * sn + smax * cs) + fabs(-D * cs + smax * sn));
    double H = (delta * Pmax / (2.0 * hmin) + 0.5 * kappa * tau) / den;
    // margin for the FP32 shadow and window start computed per pixel
    H = H * (1.0 + 1e-5) + 1e-3 * tau + 1e-6 * fmax(fabs(smin), fabs(smax));
    // (capped far above any staged range; the kernel clamps a window to the
    // staged cells, which hold every non-zero cell)
    const double Td = floor(2.0 * H / tau) + 1.0;
    const int T = den > 0.0 && Td < (double)(1 << 20) ? (int)Td : (1 << 20);
    out[t] = make_int4(cnt ? (int)lo : 0, cnt, T, __float_as_int((float)H));
    atomicMax(&maxima[0], cnt);
    atomicMax(&maxima[1], T);
}

}  // namespace

hipError_t launch_ray_tables(const double2 *views, const RayTableArgs &a, hipStream_t s) {
    const size_t n = (size_t)a.nv * a.nd;
    hipLaunchKernelGGL(ray_tables_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, views,
                       a);
    return hipGetLastError();
}

hipError_t launch_tile_table(const double2 *views, const TileTableArgs &a, int4 *out, int *maxima,
                             hipStream_t s) {
    const size_t n = (size_t)a.nv * a.tiles_x * a.tiles_y;
    hipLaunchKernelGGL(tile_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, views,
                       a, out, maxima);
    return hipGetLastError();
}

}  // namespace fanproj
