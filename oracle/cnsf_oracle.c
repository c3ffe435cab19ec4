/*
 * FP64 CPU oracle for the convolutional non-separable footprint (CNSF)
 * fan-beam projector of Zhang & Entezari, "A Convolutional Forward and
 * Back-Projection Model for Fan-Beam Geometry" (arXiv 1907.10526).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the HIP library and includes none of it.
 *
 * Everything is double precision, written as plain loops in the order the
 * paper derives the model:
 *   Sec. II-A   fan geometry: source p = D_sc u, flat detector perpendicular
 *               to u at distance D_sd from the source, detector axis
 *               R_{u perp} = [sin t, -cos t]  (Sec. III-B example).
 *   Eq. (5)-(6) pixel basis: an entry of A is the blurred projection of one
 *               translated pixel indicator.
 *   Eq. (13)    per-ray orthonormal frame (w_perp, w); s' is the signed
 *               offset of the pixel centre from the ray along w_perp.
 *   Eq. (16)    unblurred footprint = 2-direction box spline with directions
 *               zeta = R_{v(s) perp} Xi, Xi = delta * I.
 *   Eq. (17)    effective blur tau': the two bin edges, written in the ray
 *               frame, perspective-divided and scaled to the pixel depth.
 *   Eq. (18)    blurred footprint = 3-direction box spline [zeta1, zeta2, tau'].
 *   Eq. (9)     the 3-direction box spline is evaluated as the convolution of
 *               the 2-direction one with the third elementary box: the
 *               difference of the 2-direction box spline's antiderivative
 *               over the third width, divided by that width.
 *
 * Readings of passages the paper leaves open (each one is listed, with its
 * reason, in the design notes of the repository):
 *   - the blur h_tau has unit mass, so a detector value is a bin average;
 *   - the basis is centred on the pixel centre and the blur box is centred on
 *     the ray through the bin centre, so the spline is the centred one;
 *   - the perspective division of eq. (17) is taken at the depth
 *     L = w . (k - p) of the pixel centre along the ray;
 *   - a pixel of side delta is delta^2 times the unit-mass box spline M_{delta I};
 *   - a zero direction is dropped (delta distribution, Sec. IV-A);
 *   - cells outside the detector do not exist (no extrapolation).
 *
 * Parallel-beam mode (Theorem 1): every ray of a view has direction -u,
 * s' = e.k - s_m and tau' = tau.
 *
 * Arc-detector mode (the paper notes that an arc detector is a special case
 * of the same derivation, Sec. I): the cells lie on the circle of radius D_sd
 * around the source, the detector coordinate s is arc length on that circle
 * (so the ray of cell m leaves the central ray at the angle s_m / D_sd), and
 * the bin edges are the two points at s_m -/+ tau/2 on the arc.  Eq. (13),
 * (16)-(18) are then applied unchanged to that ray and those two edges.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_FAN_FLAT 0
#define ORACLE_PARALLEL 1
#define ORACLE_FAN_ARC 2

typedef struct {
    int32_t nx, ny;          /* image columns (x) and rows (y)              */
    double pixel;            /* pixel side delta                            */
    double dsc;              /* source-to-centre distance D_po              */
    double dsd;              /* source-to-detector distance D_ps            */
    int32_t n_views;
    const double *angles;    /* view angles theta_v, radians                */
    int32_t n_det;           /* detector cells                              */
    double det_spacing;      /* cell pitch Delta_s                          */
    double det_width;        /* bin width tau                               */
    int32_t mode;            /* ORACLE_FAN_FLAT, ORACLE_PARALLEL or
                                ORACLE_FAN_ARC                              */
} oracle_geom;

/* ------------------------------------------------------------------------ */
/* Box splines on the line (Sec. III-A, eq. (9)).                            */
/* ------------------------------------------------------------------------ */

/* Antiderivative (cumulative integral from -inf) of the centred box spline
 * with the two directions a <= b, i.e. of the convolution of a centred box of
 * width a with a centred box of width b, both of unit mass.  For a > 0 that
 * convolution is the trapezoid of height 1/b whose plateau spans |t| <= (b-a)/2
 * and whose support is |t| < (a+b)/2.  A zero width is a delta distribution
 * and drops out of the convolution. */
static double cdf2(double t, double a, double b)
{
    if (b == 0.0)                      /* both directions vanish: a step */
        return t >= 0.0 ? 1.0 : 0.0;
    if (a == 0.0) {                    /* one direction: a single box     */
        double h = (t + 0.5 * b) / b;
        return h <= 0.0 ? 0.0 : (h >= 1.0 ? 1.0 : h);
    }
    const double outer = 0.5 * (a + b), inner = 0.5 * (b - a);
    if (t <= -outer) return 0.0;
    if (t <= -inner) { double d = t + outer; return d * d / (2.0 * a * b); }
    if (t < inner)   return (t + 0.5 * b) / b;
    if (t < outer)   { double d = outer - t; return 1.0 - d * d / (2.0 * a * b); }
    return 1.0;
}

/* Centred, unit-mass box spline on the line with three directions of widths
 * w1, w2, w3 (absolute values are taken; a zero width is dropped).  The
 * largest width c is convolved last: M(x) = (cdf2(x + c/2) - cdf2(x - c/2)) / c,
 * which is the moving average of eq. (9) over the third direction. */
double oracle_box3(double x, double w1, double w2, double w3)
{
    double w[3] = {fabs(w1), fabs(w2), fabs(w3)};
    /* sort ascending: a = w[0] <= b = w[1] <= c = w[2] */
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (w[j] < w[i]) { double t = w[i]; w[i] = w[j]; w[j] = t; }
    const double a = w[0], b = w[1], c = w[2];
    if (c == 0.0)   /* all three directions vanish: a delta, never an entry */
        return x == 0.0 ? INFINITY : 0.0;
    return (cdf2(x + 0.5 * c, a, b) - cdf2(x - 0.5 * c, a, b)) / c;
}

/* Centred, unit-mass box spline with two directions (the unblurred footprint
 * of eq. (16)): the trapezoid itself, as the derivative of cdf2. */
double oracle_box2(double x, double w1, double w2)
{
    double a = fabs(w1), b = fabs(w2);
    if (a > b) { double t = a; a = b; b = t; }
    if (b == 0.0) return x == 0.0 ? INFINITY : 0.0;
    x = fabs(x);
    if (a == 0.0) return x < 0.5 * b ? 1.0 / b : 0.0;
    const double outer = 0.5 * (a + b), inner = 0.5 * (b - a);
    if (x >= outer) return 0.0;
    if (x <= inner) return 1.0 / b;
    return (outer - x) / (a * b);
}

/* ------------------------------------------------------------------------ */
/* Geometry (Sec. II-A, eq. (13), eq. (17)).                                 */
/* ------------------------------------------------------------------------ */

/* Centre of detector cell m along the detector axis (arc length on the arc
 * detector). */
static double cell_centre(const oracle_geom *g, int m)
{
    return ((double)m - 0.5 * (double)(g->n_det - 1)) * g->det_spacing;
}

/* Centre of pixel (i, j): columns along x, rows along y, grid centred on the
 * rotation centre. */
static void pixel_centre(const oracle_geom *g, int i, int j, double k[2])
{
    k[0] = ((double)i - 0.5 * (double)(g->nx - 1)) * g->pixel;
    k[1] = ((double)j - 0.5 * (double)(g->ny - 1)) * g->pixel;
}

/* The ray of view v through the centre of cell m: source point p, unit
 * direction w (source towards detector), unit normal w_perp = w rotated by
 * +90 degrees, and the two bin edges written in that frame (x1 along w_perp,
 * x2 along w, origin at p). */
typedef struct {
    double p[2], w[2], wp[2];
    double edge_lo[2], edge_hi[2];   /* (x1, x2) of q(s_m -/+ tau/2) - p     */
} ray_frame;

static void detector_offset(const oracle_geom *g, const double u[2], const double e[2],
                            double s, double d[2])
{
    if (g->mode == ORACLE_FAN_ARC) {
        const double gam = s / g->dsd;
        d[0] = g->dsd * (-cos(gam) * u[0] + sin(gam) * e[0]);
        d[1] = g->dsd * (-cos(gam) * u[1] + sin(gam) * e[1]);
    } else {
        d[0] = -g->dsd * u[0] + s * e[0];
        d[1] = -g->dsd * u[1] + s * e[1];
    }
}

static void make_ray(const oracle_geom *g, int v, int m, ray_frame *r)
{
    const double th = g->angles[v];
    const double u[2] = {cos(th), sin(th)};
    const double e[2] = {sin(th), -cos(th)};          /* R_{u perp}         */
    const double s = cell_centre(g, m);
    if (g->mode == ORACLE_PARALLEL) {
        /* every ray of the view runs along -u; the ray of cell m is the line
         * e.x = s_m; the frame origin is the foot of that line on e */
        r->w[0] = -u[0]; r->w[1] = -u[1];
        r->wp[0] = -r->w[1]; r->wp[1] = r->w[0];     /* = e                 */
        r->p[0] = s * e[0] + g->dsc * u[0];
        r->p[1] = s * e[1] + g->dsc * u[1];
        r->edge_lo[0] = -0.5 * g->det_width; r->edge_lo[1] = g->dsd;
        r->edge_hi[0] = 0.5 * g->det_width;  r->edge_hi[1] = g->dsd;
        return;
    }
    r->p[0] = g->dsc * u[0];
    r->p[1] = g->dsc * u[1];
    /* detector point q(s) - p: flat, -D_sd u + s e; arc, the point at angle
     * s / D_sd from -u on the circle of radius D_sd */
    double d[2];
    detector_offset(g, u, e, s, d);
    double R = sqrt(d[0] * d[0] + d[1] * d[1]);
    r->w[0] = d[0] / R; r->w[1] = d[1] / R;
    r->wp[0] = -r->w[1]; r->wp[1] = r->w[0];
    for (int side = 0; side < 2; ++side) {
        double se = s + (side ? 0.5 : -0.5) * g->det_width;
        double qe[2];
        detector_offset(g, u, e, se, qe);
        double *out = side ? r->edge_hi : r->edge_lo;
        out[0] = r->wp[0] * qe[0] + r->wp[1] * qe[1];
        out[1] = r->w[0] * qe[0] + r->w[1] * qe[1];
    }
}

/* The quantities eq. (18) is evaluated with, for the ray with frame r and the
 * pixel centred at k: sp = s' (signed offset of the pixel centre from the
 * ray), zeta1, zeta2 (the pixel directions projected on w_perp) and
 * taup = tau' (eq. (17)). */
static void terms_from_frame(const oracle_geom *g, const ray_frame *r, const double k[2],
                             double *sp, double *zeta1, double *zeta2, double *taup,
                             double *depth)
{
    const double dk[2] = {k[0] - r->p[0], k[1] - r->p[1]};
    const double s_off = r->wp[0] * dk[0] + r->wp[1] * dk[1];
    const double L = r->w[0] * dk[0] + r->w[1] * dk[1];
    *sp = s_off;
    *zeta1 = g->pixel * r->wp[0];     /* R_{v perp} xi_1, xi_1 = (delta, 0) */
    *zeta2 = g->pixel * r->wp[1];     /* R_{v perp} xi_2, xi_2 = (0, delta) */
    if (g->mode == ORACLE_PARALLEL) {
        *taup = g->det_width;
    } else {
        /* perspective division of each edge, then scaling to depth L */
        const double t_hi = r->edge_hi[0] / r->edge_hi[1];
        const double t_lo = r->edge_lo[0] / r->edge_lo[1];
        *taup = L * (t_hi - t_lo);
    }
    if (depth) *depth = L;
}

/* The same quantities for ray (v, m) and pixel (i, j). */
void oracle_entry_terms(const oracle_geom *g, int v, int m, int i, int j,
                        double *sp, double *zeta1, double *zeta2, double *taup,
                        double *depth)
{
    ray_frame r;
    make_ray(g, v, m, &r);
    double k[2];
    pixel_centre(g, i, j, k);
    terms_from_frame(g, &r, k, sp, zeta1, zeta2, taup, depth);
}

/* Matrix entry A_{(v,m),(i,j)} = delta^2 * M_[zeta1, zeta2, tau'](s'). */
double oracle_entry(const oracle_geom *g, int v, int m, int i, int j)
{
    double sp, z1, z2, tp;
    oracle_entry_terms(g, v, m, i, j, &sp, &z1, &z2, &tp, NULL);
    return g->pixel * g->pixel * oracle_box3(sp, z1, z2, tp);
}

/* Candidate cells of the pixel centred at k in the view with source direction
 * u and detector axis e: every cell whose bin meets the interval spanned by
 * the detector shadows of the pixel's four corners, widened by one extra cell
 * on each side.  The shadow of a point x is where the line from the source
 * through x meets the detector. */
static void candidate_cells_dirs(const oracle_geom *g, const double u[2], const double e[2],
                                 const double k[2], int *m_lo, int *m_hi)
{
    double smin = INFINITY, smax = -INFINITY;
    for (int c = 0; c < 4; ++c) {
        const double x = k[0] + ((c & 1) ? 0.5 : -0.5) * g->pixel;
        const double y = k[1] + ((c & 2) ? 0.5 : -0.5) * g->pixel;
        const double along = e[0] * x + e[1] * y;
        double s;
        const double depth = g->dsc - (u[0] * x + u[1] * y);
        if (g->mode == ORACLE_PARALLEL)
            s = along;
        else if (g->mode == ORACLE_FAN_ARC)
            s = g->dsd * atan2(along, depth);
        else
            s = g->dsd * along / depth;
        if (s < smin) smin = s;
        if (s > smax) smax = s;
    }
    const double half = 0.5 * (g->n_det - 1);
    const double lo = (smin - 0.5 * g->det_width) / g->det_spacing + half;
    const double hi = (smax + 0.5 * g->det_width) / g->det_spacing + half;
    long a = (long)floor(lo) - 1, b = (long)ceil(hi) + 1;
    if (a < 0) a = 0;
    if (b > g->n_det - 1) b = g->n_det - 1;
    *m_lo = (int)a;
    *m_hi = (int)b;
}

/* Candidate cells of pixel (i, j) in view v. */
static void candidate_cells(const oracle_geom *g, int v, int i, int j,
                            int *m_lo, int *m_hi)
{
    const double th = g->angles[v];
    const double u[2] = {cos(th), sin(th)};
    const double e[2] = {sin(th), -cos(th)};
    double k[2];
    pixel_centre(g, i, j, k);
    candidate_cells_dirs(g, u, e, k, m_lo, m_hi);
}

/* ------------------------------------------------------------------------ */
/* Forward and back projection (eq. (6)) and their use in SIRT.              */
/* ------------------------------------------------------------------------ */

/* y = A c.  img is [ny][nx] (x fastest), sino is [n_views][n_det].
 * dense != 0 evaluates every (ray, pixel) pair; otherwise only candidate
 * cells are visited (the two must agree exactly). */
void oracle_forward(const oracle_geom *g, const double *img, double *sino,
                    int dense)
{
    const int nv = g->n_views, nd = g->n_det;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < nv; ++v) {
        double *row = sino + (size_t)v * nd;
        for (int m = 0; m < nd; ++m) row[m] = 0.0;
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                const double c = img[(size_t)j * g->nx + i];
                int lo = 0, hi = nd - 1;
                if (!dense) candidate_cells(g, v, i, j, &lo, &hi);
                for (int m = lo; m <= hi; ++m)
                    row[m] += oracle_entry(g, v, m, i, j) * c;
            }
    }
}

/* z = A^T y. */
void oracle_back(const oracle_geom *g, const double *sino, double *img,
                 int dense)
{
    const int nx = g->nx, ny = g->ny;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double acc = 0.0;
            for (int v = 0; v < g->n_views; ++v) {
                int lo = 0, hi = g->n_det - 1;
                if (!dense) candidate_cells(g, v, i, j, &lo, &hi);
                for (int m = lo; m <= hi; ++m)
                    acc += oracle_entry(g, v, m, i, j)
                           * sino[(size_t)v * g->n_det + m];
            }
            img[(size_t)j * nx + i] = acc;
        }
}

/* One output of A c: the detector value of ray (v, m). */
double oracle_forward_ray(const oracle_geom *g, const double *img, int v, int m)
{
    double acc = 0.0;
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            int lo, hi;
            candidate_cells(g, v, i, j, &lo, &hi);
            if (m < lo || m > hi) continue;
            acc += oracle_entry(g, v, m, i, j) * img[(size_t)j * g->nx + i];
        }
    return acc;
}

/* One output of A^T y: the back-projected value of pixel (i, j). */
double oracle_back_pixel(const oracle_geom *g, const double *sino, int i, int j)
{
    double acc = 0.0;
    for (int v = 0; v < g->n_views; ++v) {
        int lo, hi;
        candidate_cells(g, v, i, j, &lo, &hi);
        for (int m = lo; m <= hi; ++m)
            acc += oracle_entry(g, v, m, i, j) * sino[(size_t)v * g->n_det + m];
    }
    return acc;
}

/* Forward projection restricted to views [v0, v1): rows v0..v1-1 of sino are
 * written (sino still points at row 0).  Used to time a bounded sample. */
void oracle_forward_views(const oracle_geom *g, const double *img, double *sino,
                          int v0, int v1)
{
    oracle_geom sub = *g;
    sub.angles = g->angles + v0;
    sub.n_views = v1 - v0;
    oracle_forward(&sub, img, sino + (size_t)v0 * g->n_det, 0);
}

/* Back projection restricted to views [v0, v1) (a partial sum over views). */
void oracle_back_views(const oracle_geom *g, const double *sino, double *img,
                       int v0, int v1)
{
    oracle_geom sub = *g;
    sub.angles = g->angles + v0;
    sub.n_views = v1 - v0;
    oracle_back(&sub, sino + (size_t)v0 * g->n_det, img, 0);
}

/* The frame of every ray, [n_views][n_det] (NULL if it cannot be allocated). */
static ray_frame *all_frames(const oracle_geom *g)
{
    const size_t nr = (size_t)g->n_views * g->n_det;
    ray_frame *f = malloc(nr * sizeof(ray_frame));
    if (!f) return NULL;
    #pragma omp parallel for schedule(static)
    for (int v = 0; v < g->n_views; ++v)
        for (int m = 0; m < g->n_det; ++m)
            make_ray(g, v, m, &f[(size_t)v * g->n_det + m]);
    return f;
}

static double entry_from_frame(const oracle_geom *g, const ray_frame *r, const double k[2])
{
    double sp, z1, z2, tp;
    terms_from_frame(g, r, k, &sp, &z1, &z2, &tp, NULL);
    return g->pixel * g->pixel * oracle_box3(sp, z1, z2, tp);
}

/* oracle_forward and oracle_back (with pruning) with every ray frame
 * (make_ray) and every view's (cos t, sin t) computed once per call instead of
 * once per entry.  The loops, the entry arithmetic and the summation order
 * are theirs, so the results are bitwise the same; only the repeated
 * evaluation of identical values is saved.  Used where full-size scans are
 * projected many times (the stored large SIRT iterate).  Each returns 0, or
 * -1 if its tables cannot be allocated. */
int oracle_forward_cached(const oracle_geom *g, const double *img, double *sino)
{
    const int nv = g->n_views, nd = g->n_det;
    ray_frame *f = all_frames(g);
    if (!f) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < nv; ++v) {
        const double th = g->angles[v];
        const double u[2] = {cos(th), sin(th)};
        const double e[2] = {sin(th), -cos(th)};
        const ray_frame *fv = f + (size_t)v * nd;
        double *row = sino + (size_t)v * nd;
        for (int m = 0; m < nd; ++m) row[m] = 0.0;
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                const double c = img[(size_t)j * g->nx + i];
                double k[2];
                pixel_centre(g, i, j, k);
                int lo, hi;
                candidate_cells_dirs(g, u, e, k, &lo, &hi);
                for (int m = lo; m <= hi; ++m)
                    row[m] += entry_from_frame(g, &fv[m], k) * c;
            }
    }
    free(f);
    return 0;
}

int oracle_back_cached(const oracle_geom *g, const double *sino, double *img)
{
    const int nx = g->nx, ny = g->ny, nv = g->n_views, nd = g->n_det;
    ray_frame *f = all_frames(g);
    double *dirs = malloc((size_t)nv * 4 * sizeof(double));
    if (!f || !dirs) { free(f); free(dirs); return -1; }
    for (int v = 0; v < nv; ++v) {
        const double th = g->angles[v];
        dirs[4 * v + 0] = cos(th); dirs[4 * v + 1] = sin(th);
        dirs[4 * v + 2] = sin(th); dirs[4 * v + 3] = -cos(th);
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double k[2];
            pixel_centre(g, i, j, k);
            double acc = 0.0;
            for (int v = 0; v < nv; ++v) {
                int lo, hi;
                candidate_cells_dirs(g, dirs + 4 * v, dirs + 4 * v + 2, k, &lo, &hi);
                const ray_frame *fv = f + (size_t)v * nd;
                for (int m = lo; m <= hi; ++m)
                    acc += entry_from_frame(g, &fv[m], k) * sino[(size_t)v * nd + m];
            }
            img[(size_t)j * nx + i] = acc;
        }
    free(f);
    free(dirs);
    return 0;
}

/* Number of (ray, pixel) pairs whose entry is non-zero. */
int64_t oracle_count_nonzero(const oracle_geom *g)
{
    int64_t total = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int v = 0; v < g->n_views; ++v)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int lo, hi;
                candidate_cells(g, v, i, j, &lo, &hi);
                for (int m = lo; m <= hi; ++m)
                    if (oracle_entry(g, v, m, i, j) != 0.0) ++total;
            }
    return total;
}

/* SIRT (simultaneous iterative reconstruction):
 *   x <- x + lambda * C .* A^T ( R .* (y - A x) ),
 *   R = 1 ./ (A 1),  C = 1 ./ (A^T 1),  with 1/0 read as 0.
 * x holds the start on entry and the iterate after `iters` steps on exit. */
void oracle_sirt(const oracle_geom *g, const double *y, double *x, int iters,
                 double lambda)
{
    const size_t np = (size_t)g->nx * g->ny, nr = (size_t)g->n_views * g->n_det;
    double *ones_img = malloc(np * sizeof(double));
    double *ones_sino = malloc(nr * sizeof(double));
    double *Rw = malloc(nr * sizeof(double));
    double *Cw = malloc(np * sizeof(double));
    double *r = malloc(nr * sizeof(double));
    double *z = malloc(np * sizeof(double));
    for (size_t k = 0; k < np; ++k) ones_img[k] = 1.0;
    for (size_t k = 0; k < nr; ++k) ones_sino[k] = 1.0;
    oracle_forward(g, ones_img, Rw, 0);
    oracle_back(g, ones_sino, Cw, 0);
    for (size_t k = 0; k < nr; ++k) Rw[k] = Rw[k] != 0.0 ? 1.0 / Rw[k] : 0.0;
    for (size_t k = 0; k < np; ++k) Cw[k] = Cw[k] != 0.0 ? 1.0 / Cw[k] : 0.0;
    for (int it = 0; it < iters; ++it) {
        oracle_forward(g, x, r, 0);
        for (size_t k = 0; k < nr; ++k) r[k] = Rw[k] * (y[k] - r[k]);
        oracle_back(g, r, z, 0);
        for (size_t k = 0; k < np; ++k) x[k] += lambda * Cw[k] * z[k];
    }
    free(ones_img); free(ones_sino); free(Rw); free(Cw); free(r); free(z);
}

/* Threads the OpenMP loops use (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
