// The reference projector of the paper's experiments (Sec. V, "Ref"): the
// exact entry of a pixel on a cell, i.e. the exact length of the ray through
// the pixel, averaged over the cell's detector coordinate (eq. (2)-(3) with the
// unit-mass blur), without the effective-blur approximation of eq. (17).
// Everything in FP64.  Slow by design: it is the yardstick the CNSF kernels
// are measured against (single-pixel profiles, maximum errors, image-level
// errors, reconstructions from reference data), not a production path.
//
// The chord of a ray through a pixel is a smooth function of the detector
// coordinate u between the coordinates of the rays through the pixel's four
// corners, so the average over the cell is integrated exactly up to rounding
// by Gauss-Legendre quadrature on each piece between those breakpoints.
//
// Detector coordinate u of a ray, per beam:
//   flat      ray from the source p = D_sc (cos t, sin t) through the detector
//             point p - D_sd u_vec + u e,   e = (sin t, -cos t);
//   arc       ray from the source at angle u / D_sd from -u_vec towards e;
//   parallel  the line e . x = u, direction -u_vec.
#include <algorithm>
#include <cmath>

#include "fanproj_internal.h"

namespace fanproj {
namespace {

constexpr int kRefMaxQuad = 24;
constexpr int kRefThreads = 128;

struct RefArgs {
    int nx, ny, nv, nd, beam, nq;
    double pixel, dsc, dsd, pitch, width;
    double gl_x[kRefMaxQuad], gl_w[kRefMaxQuad];   // nodes and weights on [-1, 1]
};

// Ray of detector coordinate u: a point on it and its unit direction.
__device__ void ref_ray(const RefArgs &a, double cs, double sn, double u, double &ox, double &oy,
                        double &dx, double &dy) {
    if (a.beam == FP_PARALLEL) {
        ox = u * sn + a.dsc * cs;
        oy = -u * cs + a.dsc * sn;
        dx = -cs;
        dy = -sn;
        return;
    }
    ox = a.dsc * cs;
    oy = a.dsc * sn;
    if (a.beam == FP_FAN_ARC) {
        double sg, cg;
        sincos(u / a.dsd, &sg, &cg);
        dx = -cg * cs + sg * sn;
        dy = -cg * sn - sg * cs;
    } else {
        const double qx = -a.dsd * cs + u * sn, qy = -a.dsd * sn - u * cs;
        const double r = sqrt(qx * qx + qy * qy);
        dx = qx / r;
        dy = qy / r;
    }
}

// Detector coordinate of the ray through the point (x, y).
__device__ double ref_coord(const RefArgs &a, double cs, double sn, double x, double y) {
    const double along = sn * x - cs * y;
    if (a.beam == FP_PARALLEL) return along;
    const double depth = a.dsc - (cs * x + sn * y);
    if (a.beam == FP_FAN_ARC) return a.dsd * atan2(along, depth);
    return a.dsd * along / depth;
}

// Length of the line (ox, oy) + t (dx, dy), t unbounded, inside the box.
__device__ double ref_chord(double ox, double oy, double dx, double dy, double bx0, double bx1,
                            double by0, double by1) {
    double t0 = -INFINITY, t1 = INFINITY;
    if (dx != 0.0) {
        const double ta = (bx0 - ox) / dx, tb = (bx1 - ox) / dx;
        t0 = fmax(t0, fmin(ta, tb));
        t1 = fmin(t1, fmax(ta, tb));
    } else if (ox < bx0 || ox > bx1) {
        return 0.0;
    }
    if (dy != 0.0) {
        const double ta = (by0 - oy) / dy, tb = (by1 - oy) / dy;
        t0 = fmax(t0, fmin(ta, tb));
        t1 = fmin(t1, fmax(ta, tb));
    } else if (oy < by0 || oy > by1) {
        return 0.0;
    }
    return fmax(0.0, t1 - t0);
}

// Exact entry of pixel (i, j) on cell m of the view (cs, sn).
__device__ double ref_entry(const RefArgs &a, double cs, double sn, int m, int i, int j) {
    const double d = a.pixel;
    const double kx = (i - 0.5 * (a.nx - 1)) * d, ky = (j - 0.5 * (a.ny - 1)) * d;
    const double bx0 = kx - 0.5 * d, bx1 = kx + 0.5 * d, by0 = ky - 0.5 * d, by1 = ky + 0.5 * d;
    const double sm = (m - 0.5 * (a.nd - 1)) * a.pitch;
    const double lo = sm - 0.5 * a.width, hi = sm + 0.5 * a.width;
    double c[4] = {ref_coord(a, cs, sn, bx0, by0), ref_coord(a, cs, sn, bx1, by0),
                   ref_coord(a, cs, sn, bx0, by1), ref_coord(a, cs, sn, bx1, by1)};
    // sort the four corner coordinates
    for (int p = 1; p < 4; ++p)
        for (int q = p; q > 0 && c[q] < c[q - 1]; --q) {
            const double t = c[q];
            c[q] = c[q - 1];
            c[q - 1] = t;
        }
    if (!(hi > c[0] && lo < c[3])) return 0.0;   // the cell misses the pixel's shadow
    double cuts[6];
    int nc = 0;
    cuts[nc++] = fmax(lo, c[0]);
    for (int p = 0; p < 4; ++p)
        if (c[p] > cuts[0] && c[p] < fmin(hi, c[3])) cuts[nc++] = c[p];
    cuts[nc++] = fmin(hi, c[3]);
    double total = 0.0;
    for (int p = 0; p + 1 < nc; ++p) {
        const double s0 = cuts[p], s1 = cuts[p + 1];
        if (!(s1 > s0)) continue;
        const double half = 0.5 * (s1 - s0), mid = 0.5 * (s1 + s0);
        double seg = 0.0;
        for (int q = 0; q < a.nq; ++q) {
            double ox, oy, dx, dy;
            ref_ray(a, cs, sn, fma(half, a.gl_x[q], mid), ox, oy, dx, dy);
            seg = fma(a.gl_w[q], ref_chord(ox, oy, dx, dy, bx0, bx1, by0, by1), seg);
        }
        total = fma(half, seg, total);
    }
    return total / a.width;
}

// Forward: thread = ray (view blockIdx.y, cell m).  The rays of the cell
// sweep a wedge (a strip for parallel beams) between the two edge rays; the
// thread walks the image axis closest to the central ray and, per row, the
// pixels the wedge can meet there.
__global__ __launch_bounds__(kRefThreads) void ref_forward_kernel(RefArgs a,
                                                                  const double2 *__restrict__ views,
                                                                  const double *__restrict__ img,
                                                                  double *__restrict__ sino) {
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int v = (int)blockIdx.y;
    if (m >= a.nd) return;
    const double cs = views[v].x, sn = views[v].y, d = a.pixel;
    const double sm = (m - 0.5 * (a.nd - 1)) * a.pitch;
    double ex[2][2], ey[2][2];   // [edge][point, direction]
    double cx, cy, cdx, cdy;
    ref_ray(a, cs, sn, sm, cx, cy, cdx, cdy);
    for (int k = 0; k < 2; ++k)
        ref_ray(a, cs, sn, sm + (k ? 0.5 : -0.5) * a.width, ex[k][0], ey[k][0], ex[k][1], ey[k][1]);
    const bool by_rows = fabs(cdy) >= fabs(cdx);
    const int nr = by_rows ? a.ny : a.nx, nq = by_rows ? a.nx : a.ny;
    const double r0 = -0.5 * ((by_rows ? a.ny : a.nx) - 1) * d;   // centre of row 0
    const double q0 = -0.5 * (nq - 1) * d;                         // centre of column 0
    double acc = 0.0;
    for (int r = 0; r < nr; ++r) {
        // cross-axis extent of the wedge inside the band of row r
        double qmin = INFINITY, qmax = -INFINITY;
        for (int k = 0; k < 2; ++k)
            for (int side = 0; side < 2; ++side) {
                const double rb = r0 + (r + (side ? 0.5 : -0.5)) * d;
                const double px = by_rows ? ex[k][0] : ey[k][0], pr = by_rows ? ey[k][0] : ex[k][0];
                const double dq = by_rows ? ex[k][1] : ey[k][1], dr = by_rows ? ey[k][1] : ex[k][1];
                const double q = px + (rb - pr) * dq / dr;
                qmin = fmin(qmin, q);
                qmax = fmax(qmax, q);
            }
        const double flo = (qmin - q0) / d - 0.5, fhi = (qmax - q0) / d + 0.5;
        if (!(fhi >= 0.0) || !(flo <= nq - 1.0)) continue;
        const int i0 = max((int)floor(fmax(flo, -1.0)), 0);
        const int i1 = min((int)ceil(fmin(fhi, (double)nq)), nq - 1);
        for (int q = i0; q <= i1; ++q) {
            const int i = by_rows ? q : r, j = by_rows ? r : q;
            const double c = img[(size_t)j * a.nx + i];
            if (c != 0.0) acc = fma(ref_entry(a, cs, sn, m, i, j), c, acc);
        }
    }
    sino[(size_t)v * a.nd + m] = acc;
}

// Back (the exact adjoint, same entries): thread = pixel; per view, the cells
// whose width overlaps the pixel's shadow.
__global__ __launch_bounds__(kRefThreads) void ref_back_kernel(RefArgs a,
                                                               const double2 *__restrict__ views,
                                                               const double *__restrict__ sino,
                                                               double *__restrict__ img) {
    const int pix = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (pix >= a.nx * a.ny) return;
    const int i = pix % a.nx, j = pix / a.nx;
    const double d = a.pixel, c0 = 0.5 * (a.nd - 1);
    const double kx = (i - 0.5 * (a.nx - 1)) * d, ky = (j - 0.5 * (a.ny - 1)) * d;
    double acc = 0.0;
    for (int v = 0; v < a.nv; ++v) {
        const double cs = views[v].x, sn = views[v].y;
        double cmin = INFINITY, cmax = -INFINITY;
        for (int k = 0; k < 4; ++k) {
            const double c = ref_coord(a, cs, sn, kx + ((k & 1) ? 0.5 : -0.5) * d,
                                       ky + ((k & 2) ? 0.5 : -0.5) * d);
            cmin = fmin(cmin, c);
            cmax = fmax(cmax, c);
        }
        const int m0 = max((int)floor((cmin - 0.5 * a.width) / a.pitch + c0), 0);
        const int m1 = min((int)ceil((cmax + 0.5 * a.width) / a.pitch + c0), a.nd - 1);
        for (int m = m0; m <= m1; ++m) {
            const double y = sino[(size_t)v * a.nd + m];
            if (y != 0.0) acc = fma(ref_entry(a, cs, sn, m, i, j), y, acc);
        }
    }
    img[pix] = acc;
}

// Gauss-Legendre nodes and weights on [-1, 1]: roots of P_n by Newton's
// method from the usual cosine starting points, weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double *x, double *w) {
    for (int k = 0; k < n; ++k) {
        double z = std::cos(M_PI * (k + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int l = 2; l <= n; ++l) {
                const double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(z), p0 = P_{n-1}(z)
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[k] = z;
        w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

RefArgs ref_args(const fp_geometry *g, int nq) {
    RefArgs a{};
    a.nx = g->nx; a.ny = g->ny; a.nv = g->nv; a.nd = g->nd; a.beam = g->beam; a.nq = nq;
    a.pixel = g->pixel; a.dsc = g->dsc; a.dsd = g->dsd; a.pitch = g->pitch; a.width = g->tau;
    gauss_legendre(nq, a.gl_x, a.gl_w);
    return a;
}

}  // namespace

hipError_t launch_reference(const fp_geometry *g, bool forward, const double *in, double *out,
                            int batch, int quad, hipStream_t s) {
    const RefArgs a = ref_args(g, std::min(std::max(quad, 1), kRefMaxQuad));
    const size_t np = (size_t)g->nx * g->ny, nr = (size_t)g->nv * g->nd;
    for (int b = 0; b < batch; ++b) {
        if (forward) {
            dim3 grid((g->nd + kRefThreads - 1) / kRefThreads, g->nv);
            hipLaunchKernelGGL(ref_forward_kernel, grid, dim3(kRefThreads), 0, s, a, g->dev.views,
                               in + b * np, out + b * nr);
        } else {
            dim3 grid((unsigned)((np + kRefThreads - 1) / kRefThreads));
            hipLaunchKernelGGL(ref_back_kernel, grid, dim3(kRefThreads), 0, s, a, g->dev.views,
                               in + b * nr, out + b * np);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace fanproj
