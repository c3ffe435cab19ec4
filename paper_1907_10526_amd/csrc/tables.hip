// Geometry tables built on the device (FP64 arithmetic): the per-ray
// constants of eq. (13), (16), (17) and the per-(view, tile) cell ranges and
// window bounds of the back projection.  One thread per ray and one per
// (view, tile); the host supplies only the per-view cosines and sines.
#include "fanproj_internal.h"
#include "tables.h"

namespace fanproj {
namespace {

// Unit normal w_perp of the ray of cell m (w rotated by +90 degrees, w from
// the source towards the detector), the blur constant ghr and 1/R.  The back
// projection's tables are these constants in units of R for the flat
// detector (its s' R and R L are exact numerators, see RayTables).
//   flat:     w_perp = (D e + s u) / R, R = sqrt(D^2 + s^2); eq. (17) gives
//             tau' = g L with g = (tau/2) D [1/(D^2 + s(s + tau/2)) +
//             1/(D^2 + s(s - tau/2))], stored as ghr = g / (2R) (the kernels
//             form R L exactly and multiply);
//   arc:      w_perp = cos(g) e + sin(g) u at g = s / D; tau' = 2 tan(tau/(2D)) L,
//             stored as ghr = tan(tau / (2D)) (the kernels form L);
//   parallel: w_perp = e; tau' = tau, stored as ghr = tau / 2.
struct RayFrame {
    double wpx, wpy, inv_r, ghr;
};

__device__ RayFrame ray_frame(int beam, double cs, double sn, double s, double D, double tau) {
    RayFrame f;
    if (beam == FP_PARALLEL) {
        f.wpx = sn;
        f.wpy = -cs;
        f.inv_r = 1.0;
        f.ghr = 0.5 * tau;
    } else if (beam == FP_FAN_ARC) {
        double sg, cg;
        sincos(s / D, &sg, &cg);
        f.wpx = cg * sn + sg * cs;
        f.wpy = -cg * cs + sg * sn;
        f.inv_r = cg / D;
        f.ghr = tan(0.5 * tau / D);
    } else {
        const double R = sqrt(D * D + s * s);
        f.wpx = (D * sn + s * cs) / R;
        f.wpy = (-D * cs + s * sn) / R;
        f.inv_r = 1.0 / R;
        const double gm = 0.5 * tau * D *
                          (1.0 / (D * D + s * (s + 0.5 * tau)) + 1.0 / (D * D + s * (s - 0.5 * tau)));
        f.ghr = gm / (2.0 * R);
    }
    return f;
}

__global__ __launch_bounds__(256) void ray_tables_kernel(const double2 *__restrict__ views,
                                                         RayTableArgs a) {
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (size_t)a.nv * a.nd) return;
    const int v = (int)(r / a.nd), m = (int)(r % a.nd);
    const double delta = a.pixel;
    const double s = (m - 0.5 * (a.nd - 1)) * a.pitch;
    const RayFrame f = ray_frame(a.beam, views[v].x, views[v].y, s, a.dsd, a.width);
    // projected pixel widths a <= b (eq. (16))
    const double z1 = delta * fabs(f.wpx), z2 = delta * fabs(f.wpy);
    const double lo = fmin(z1, z2), hi = fmax(z1, z2);
    const double a_safe = fmax(lo, 1e-30);
    // the back projection's scale: R_m for the flat detector, 1 otherwise
    const double Rs = a.beam == FP_FAN_FLAT ? 1.0 / f.inv_r : 1.0;
    const double val[kRayTables] = {
        f.ghr,                         // ghr
        0.5 * (lo + hi),               // hab
        1.0 / a_safe,                  // ia
        -0.5 * (hi - lo) / a_safe,     // nhbia
        0.5 * lo,                      // ha
        delta * delta / (2.0 * hi),    // wb
        f.ghr * Rs,                    // bgh
        0.5 * (lo + hi) * Rs,          // bhab
        1.0 / (a_safe * Rs),           // bia
        0.5 * lo * Rs,                 // bha
        delta * delta / (2.0 * hi) / (f.ghr * Rs),   // bwg
    };
    // The kernels form u = clamp(m / a + nhbia) with m <= hab, which is 1 in
    // exact arithmetic at m = hab: nhbia is raised by the few ulps that make
    // the rounded FMA reach 1 there for both the forward's and the back
    // projection's constants, so that an entry outside the footprint's
    // support is exactly zero (the SIRT weights invert the row and column
    // sums).  With a = 0 the term u multiplies is zero and nothing is needed.
    float nh32 = (float)val[3];
    double nh64 = val[3];
    if (lo > 0.0) {
        const float h1 = (float)val[1], i1 = (float)val[2], h2 = (float)val[7], i2 = (float)val[8];
        for (int k = 0; k < 16 && (fmaf(h1, i1, nh32) < 1.0f || fmaf(h2, i2, nh32) < 1.0f); ++k)
            nh32 = nextafterf(nh32, INFINITY);
        for (int k = 0; k < 16 && (fma(val[1], val[2], nh64) < 1.0 || fma(val[7], val[8], nh64) < 1.0); ++k)
            nh64 = nextafter(nh64, INFINITY);
    }
#pragma unroll
    for (int k = 0; k < kRayTables; ++k) {
        if (a.f32[k]) a.f32[k][r] = k == 3 ? nh32 : (float)val[k];
        if (a.f64[k]) a.f64[k][r] = k == 3 ? nh64 : val[k];
    }
}

// Largest |cos psi| + |sin psi| over psi in [p0, p1] (its peaks, sqrt 2, sit
// at pi/4 + k pi/2).
__device__ double pmax_interval(double p0, double p1) {
    const double q = 0.5 * M_PI;
    if (floor((p1 - 0.25 * M_PI) / q) >= ceil((p0 - 0.25 * M_PI) / q)) return sqrt(2.0);
    return fmax(fabs(cos(p0)) + fabs(sin(p0)), fabs(cos(p1)) + fabs(sin(p1)));
}

// Cells that any pixel of a back-projection tile can touch.  A non-zero
// entry needs the ray through the cell centre to pass within hab + hc of the
// pixel centre, i.e. to cross the pixel dilated by hc <= hc_max; so the ray
// crosses the tile rectangle dilated by hc_max, whose detector shadow is
// spanned by its corners.  One guard cell on each side.
//
// Window of one pixel k: its non-zero cells lie within H of the pixel's own
// coordinate (flat: its shadow s_k = D (e.k) / h_k; parallel: e.k; arc: its
// angle g_k = atan2(e.k, h_k)), in the units of that coordinate.
//
// Flat: from s' = h (s_k - s_m) / R_m and the support |s'| < hab + hc: the
// pixel term hab R / h equals delta P(s_m) / (2h) with
// P(s) = |D sin + s cos| + |-D cos + s sin| (Lipschitz constant sqrt 2); the
// blur term hc R / h is at most kappa tau/2 (1 + |s_m - s_k| / (2D)),
// kappa = 1 / (1 - tau^2 / (16 D^2)).  Solved for |s_m - s_k|:
//   H_k = (delta P(s_k) / (2 h_k) + kappa tau / 2) / (1 - delta / (sqrt2 h_k) - kappa tau / (4D)).
// Over a tile P(s_k) is largest at an end of the tile's shadow (P is convex)
// and h_k smallest at a corner, which bounds H_k by H_tile.
//
// Parallel: |e.k - s_m| < hab + tau/2 with hab = delta (|sin| + |cos|) / 2.
//
// Arc: s' = rho sin(g_k - g_m) and hc = tan(tau/(2D)) rho cos(g_k - g_m), rho the
// distance of the pixel centre from the source, so a non-zero entry needs
// |g_k - g_m| < tau/(2D) + asin(hab / rho), with rho >= h >= the tile's
// smallest depth and hab = delta P(psi) / 2 at the direction psi of w_perp.
//
// The window of every pixel of the tile then holds T = floor(2 H / step) + 1
// cells, step the cell spacing in the same coordinate; the table stores the
// constant that places it (see below) rather than H.
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
    const double D = a.dsd, tau = a.width, delta = a.pixel, c0 = 0.5 * (a.nd - 1);
    const double x0 = -0.5 * (a.nx - 1) * delta, y0 = -0.5 * (a.ny - 1) * delta;
    const int i0 = tx * kBackTileW, i1 = min(a.nx, i0 + kBackTileW) - 1;
    const int j0 = ty * kBackTileH, j1 = min(a.ny, j0 + kBackTileH) - 1;
    const double ex[2] = {x0 + (i0 - 0.5) * delta, x0 + (i1 + 0.5) * delta};
    const double ey[2] = {y0 + (j0 - 0.5) * delta, y0 + (j1 + 0.5) * delta};
    // the coordinate of a point x in which cells are evenly spaced by `step`
    const int beam = a.beam;
    const double step = beam == FP_FAN_ARC ? a.pitch / D : a.pitch;
    auto coord = [&](double x, double y, double depth) {
        const double along = sn * x - cs * y;
        if (beam == FP_PARALLEL) return along;
        if (beam == FP_FAN_ARC) return atan2(along, depth);
        return D * along / depth;
    };
    double smin = INFINITY, smax = -INFINITY, hmin = INFINITY;
    double dmin = INFINITY, dmax = -INFINITY;
    bool in_front = true;
    for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy) {
            const double x = ex[cx], y = ey[cy];
            const double depth = a.dsc - (cs * x + sn * y);
            hmin = fmin(hmin, depth);
            const double sh = coord(x, y, depth);
            smin = fmin(smin, sh);
            smax = fmax(smax, sh);
            const double xd = x + (cx ? a.hc_max : -a.hc_max), yd = y + (cy ? a.hc_max : -a.hc_max);
            const double dd = a.dsc - (cs * xd + sn * yd);
            if (beam != FP_PARALLEL && !(dd > 0.0)) in_front = false;
            const double shd = coord(xd, yd, dd);
            dmin = fmin(dmin, shd);
            dmax = fmax(dmax, shd);
        }
    long lo = 0, hi = a.nd - 1;
    if (in_front) {
        lo = max((long)ceil(dmin / step + c0) - 1, 0L);
        hi = min((long)floor(dmax / step + c0) + 1, (long)a.nd - 1);
    }
    const int cnt = hi >= lo ? (int)(hi - lo + 1) : 0;
    double H;
    bool ok = true;
    if (beam == FP_PARALLEL) {
        H = 0.5 * delta * (fabs(sn) + fabs(cs)) + 0.5 * tau;
    } else if (beam == FP_FAN_ARC) {
        const double b0 = 0.5 * tau / D;
        const double H0 = b0 + asin(fmin(1.0, delta / (sqrt(2.0) * hmin)));
        // w_perp of the ray at angle g points along psi = t - pi/2 + g
        const double psi0 = atan2(-cs, sn);
        const double P = pmax_interval(psi0 + smin - H0, psi0 + smax + H0);
        H = b0 + asin(fmin(1.0, 0.5 * delta * P / hmin));
        ok = hmin > 0.0;
    } else {
        const double kappa = 1.0 / (1.0 - tau * tau / (16.0 * D * D));
        const double den = 1.0 - delta / (sqrt(2.0) * hmin) - kappa * tau / (4.0 * D);
        const double Pmax = fmax(fabs(D * sn + smin * cs) + fabs(-D * cs + smin * sn),
                                 fabs(D * sn + smax * cs) + fabs(-D * cs + smax * sn));
        H = (delta * Pmax / (2.0 * hmin) + 0.5 * kappa * tau) / den;
        ok = den > 0.0;
    }
    // margin for the FP32 coordinate and window start computed per pixel,
    // including the FP32 rounding of the window constant below
    const int M0 = cnt ? (int)lo : 0;
    const double rel = (double)M0 - kBackPad - c0;   // staged cell 0 from the centre, in cells
    H = H * (1.0 + 1e-5) + 1e-3 * step + 1e-6 * fmax(fabs(smin), fabs(smax)) +
        (beam == FP_FAN_ARC ? 1e-7 : 0.0) + ldexp(fabs(rel) + 2.0, -21) * step;
    // (capped far above any staged range; the kernel clamps a window to the
    // staged cells, which hold every non-zero cell)
    const double Td = floor(2.0 * H / step) + 1.0;
    const int T = ok && Td < (double)(1 << 20) ? (int)Td : (1 << 20);
    // A pixel with coordinate c_k starts its window at staged cell
    // floor((c_k - H) / step + c0) + 1 - (M0 - kBackPad) = floor(c_k / step + wc):
    // the first cell past c_k - H, and every non-zero cell lies past it.
    const float wc = (float)(-H / step - rel + 1.0);
    out[t] = make_int4(M0, cnt, T, __float_as_int(wc));
    // (the maxima only grow, so a value no larger than one already read needs
    // no atomic: most threads skip it instead of all contending for two
    // addresses)
    if (cnt > __hip_atomic_load(&maxima[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&maxima[0], cnt);
    if (T > __hip_atomic_load(&maxima[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&maxima[1], T);
}

__global__ __launch_bounds__(256) void arc_cells_kernel(int nd, double pitch, double dsd,
                                                        double2 *__restrict__ cells,
                                                        float2 *__restrict__ rot,
                                                        double2 *__restrict__ rot64) {
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    double sg, cg;
    if (k < kBackMaxUnrolled) {
        sincos(k * (pitch / dsd), &sg, &cg);
        rot[k] = make_float2((float)cg, (float)sg);
        rot64[k] = make_double2(cg, sg);
    }
    if (k >= nd + 2 * kBackPad) return;
    const int m = k - kBackPad;
    sincos((m - 0.5 * (nd - 1)) * pitch / dsd, &sg, &cg);
    cells[k] = make_double2(cg, sg);
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

hipError_t launch_arc_cells(int nd, double pitch, double dsd, double2 *cells, float2 *rot,
                            double2 *rot64, hipStream_t s) {
    const int n = nd + 2 * kBackPad;   // > kBackMaxUnrolled
    hipLaunchKernelGGL(arc_cells_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nd,
                       pitch, dsd, cells, rot, rot64);
    return hipGetLastError();
}

}  // namespace fanproj
