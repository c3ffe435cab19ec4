/*
 * fanproj: fan-beam forward and back-projection with the convolutional
 * non-separable footprint (CNSF) of Zhang & Entezari, "A Convolutional
 * Forward and Back-Projection Model for Fan-Beam Geometry" (arXiv 1907.10526),
 * on AMD Instinct MI355X (gfx950).
 *
 * The system matrix A is never stored (the paper's "on-the-fly, memory-less"
 * operator, Sec. V-C).  Entry A_{(v,m),k} is the detector-blurred projection of
 * the indicator of pixel k on the cell m of view v, in closed form (Sec. IV,
 * eq. (18)):
 *     A = delta^2 * M_[zeta1, zeta2, tau'](s'),
 * a centred, unit-mass, 3-direction box spline whose directions are the two
 * pixel edges projected perpendicular to the ray through the cell centre
 * (eq. (16)) and the effective blur tau' (eq. (17)): the cell's two edges seen
 * from the source, perspective-divided and scaled to the pixel's depth along
 * that ray.  s' is the signed distance of the pixel centre from the ray.
 *
 * Geometry (Sec. II-A): view angle t puts the source at
 * D_sc * (cos t, sin t); the flat detector is perpendicular to that direction
 * at distance D_sd from the source; its axis is (sin t, -cos t) (the
 * projection R_{u perp} = [sin t, -cos t] of Sec. III-B).  Cell m is centred at
 * s_m = (m - (n_det - 1)/2) * pitch on that axis, with pitch = det_width for
 * fp_geometry_create.  Pixel (i, j) of an nx x ny image is centred at
 * ((i - (nx-1)/2) delta, (j - (ny-1)/2) delta): columns run along x, rows
 * along y.  fp_geometry_create_desc adds the variants the derivation covers:
 * an arc detector, parallel beams and a pitch different from the width.
 *
 * Layouts (device memory, FP32, contiguous):
 *     image    [batch][ny][nx]          x fastest
 *     sinogram [batch][n_views][n_det]  detector cell fastest
 *
 * Precision: footprint arithmetic and accumulation in FP32; per-view fan
 * geometry and the pixel-to-ray offsets in FP64 (Sec. IV's closed form is
 * evaluated in a cancellation-free form, so no FP64 is needed inside it).
 *
 * Threading and streams: every call is asynchronous on `stream` (a
 * hipStream_t; NULL means the legacy default stream) and returns after
 * launching.  A geometry is immutable after creation apart from the SIRT
 * weights, which the first fp_sirt_step builds once (guarded); any number of
 * threads and streams may then share it.  Kernel faults surface at the
 * caller's next synchronisation, or as FP_ERR_DEVICE from a later call.
 *
 * Scratch: the launches' temporary buffers (padded image copies, view-group
 * partial sums) come from per-device buffers the library keeps for the life
 * of the process and reuses across calls, streams and threads; each reuse is
 * ordered on the device after the buffer's previous use by an event, so
 * calls do not wait on the host.  A buffer grows (after its last use has
 * finished) when a call needs more than it holds.
 *
 * Errors: no exception crosses this interface.  Every function returns an
 * fp_status; for a non-OK status fp_last_error() gives a message (per calling
 * thread).  Outputs are left untouched when arguments are rejected.
 */
#ifndef FANPROJ_H
#define FANPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FP_OK = 0,
    FP_ERR_INVALID_ARG = 1,   /* null pointer, size < 1, non-finite value,
                                 geometry with a pixel at or behind the source */
    FP_ERR_OUT_OF_MEMORY = 2, /* a device allocation failed                    */
    FP_ERR_DEVICE = 3,        /* a HIP call or kernel launch failed            */
    FP_ERR_UNSUPPORTED = 4    /* valid but beyond the library's limits         */
} fp_status;

typedef struct fp_geometry fp_geometry;   /* opaque */

/* Create a fan-beam geometry on the current HIP device (Sec. II-A; the
 * parameter set of Sec. V: image grid, pixel size, source-to-centre and
 * source-to-detector distances, view angles, detector count, cell width).
 *
 *   nx, ny               image columns and rows, >= 1
 *   pixel_size           delta > 0
 *   dist_source_center   D_sc; must exceed delta * (sqrt(nx^2 + ny^2)/2 + 1)
 *                        so that every pixel lies in front of the source
 *   dist_source_detector D_sd > D_sc (the detector lies beyond the centre)
 *   n_views, view_angles host array of n_views finite angles in radians; it
 *                        is copied, the caller keeps ownership
 *   n_det, det_width     cell count >= 1 and width (= pitch) > 0
 *   out                  receives the handle; release it with
 *                        fp_geometry_destroy
 *
 * The per-view and per-ray tables are computed on the host in FP64 and copied
 * to the device once; the call synchronises with the device.  Returns
 * FP_ERR_INVALID_ARG for the cases above, FP_ERR_OUT_OF_MEMORY if the tables
 * do not fit, FP_ERR_UNSUPPORTED if the geometry needs more on-chip memory
 * per work-group than the kernels are built for (very narrow cells). */
fp_status fp_geometry_create(int32_t nx, int32_t ny, double pixel_size,
                             double dist_source_center,
                             double dist_source_detector, int32_t n_views,
                             const double *view_angles, int32_t n_det,
                             double det_width, fp_geometry **out);

/* Beam and detector shapes of fp_geometry_create_desc. */
typedef enum {
    /* fan beam, flat detector: as fp_geometry_create */
    FP_FAN_FLAT = 0,
    /* fan beam, arc detector: the cells lie on the circle of radius D_sd
     * around the source and s is arc length on it, so the ray of cell m
     * leaves the central ray (from the source through the centre) at the
     * angle s_m / D_sd, towards +(sin t, -cos t) for s_m > 0; the cell's two
     * edges are the points at s_m -/+ width/2 on the arc.  The paper notes
     * the arc detector as a special case of its flat-detector derivation
     * (Sec. I); eq. (13), (16)-(18) are applied to that ray and those edges,
     * which gives tau' = L * 2 tan(width / (2 D_sd)). */
    FP_FAN_ARC = 1,
    /* parallel beam: every ray of view t runs along -(cos t, sin t); the ray
     * of cell m is the line (sin t, -cos t) . x = s_m and tau' = width, for
     * which the model is exact (Theorem 1).  The two distances are ignored. */
    FP_PARALLEL = 2
} fp_beam;

/* Full geometry description for fp_geometry_create_desc.  Fields as for
 * fp_geometry_create, plus:
 *   beam       an fp_beam value
 *   det_pitch  distance between neighbouring cell centres (> 0); cells may
 *              overlap (width > pitch) or leave gaps (width < pitch), the
 *              separate spacing and width of Sec. V
 *   det_width  the width tau of one cell's aperture (> 0)
 * For FP_PARALLEL, dist_source_center and dist_source_detector are not read.
 * For FP_FAN_ARC, the outermost cell edge must stay within 80 degrees of the
 * central ray: (n_det/2) * det_pitch + det_width/2 < 1.396 * D_sd. */
typedef struct {
    int32_t beam;
    int32_t nx, ny;
    double pixel_size;
    double dist_source_center;
    double dist_source_detector;
    int32_t n_views;
    const double *view_angles;   /* host, n_views finite radians, copied */
    int32_t n_det;
    double det_pitch;
    double det_width;
} fp_geometry_desc;

/* Create a geometry from a description; otherwise exactly as
 * fp_geometry_create (same validation, errors, ownership and
 * synchronisation).  fp_geometry_create(...) is fp_geometry_create_desc with
 * beam = FP_FAN_FLAT and det_pitch = det_width.  Every other entry point
 * accepts a geometry of any beam. */
fp_status fp_geometry_create_desc(const fp_geometry_desc *desc, fp_geometry **out);

/* Release the geometry.  The call does not wait: its device memory (tables,
 * SIRT weights) goes to a per-device list of idle blocks that later
 * geometries reuse only after the work this library queued with it (the
 * latest launches on every stream that used it) has completed; idle blocks
 * beyond 1 GiB per device are freed, after that work.  The handle is invalid
 * on return.  fp_sirt_step_noalloc calls are not tracked: a caller that
 * destroys a geometry with such calls still queued must synchronise first.
 * NULL is a no-op. */
fp_status fp_geometry_destroy(fp_geometry *g);

/* Forward projection y = A c (eq. (6)): for every image of the batch, every
 * view and every cell, the sum over pixels of the CNSF entry times the pixel
 * coefficient.
 *   image  device, [batch][ny][nx], read only
 *   sino   device, [batch][n_views][n_det], overwritten (no accumulation)
 *   batch  >= 1
 * The two buffers must not overlap.  Each output is written exactly once by
 * one thread; results are bitwise reproducible run to run. */
fp_status fp_forward(const fp_geometry *g, const float *image, float *sino,
                     int32_t batch, void *stream);

/* Back projection z = A^T y, the exact adjoint of fp_forward (same entries):
 *   sino   device, [batch][n_views][n_det], read only
 *   image  device, [batch][ny][nx], overwritten
 * Gather form: each pixel sums its own entries over all views; no atomics,
 * bitwise reproducible. */
fp_status fp_back(const fp_geometry *g, const float *sino, float *image,
                  int32_t batch, void *stream);

/* FP64 instantiations of fp_forward and fp_back: the same kernels, entry
 * arithmetic and accumulation in double precision, with the per-ray
 * constants in double precision (built on the device by the first FP64 call,
 * which synchronises).  Layouts, ownership and errors as for the FP32 calls;
 * FP_ERR_UNSUPPORTED if the back projection's per-tile cell staging does not
 * fit on chip in FP64.  Meant for checks that need more than FP32 (finite
 * differences, adjoint identities), not for throughput. */
fp_status fp_forward_f64(const fp_geometry *g, const double *image, double *sino,
                         int32_t batch, void *stream);
fp_status fp_back_f64(const fp_geometry *g, const double *sino, double *image,
                      int32_t batch, void *stream);

/* The reference projector of the paper's experiments (Sec. V): entry
 * (v, m, k) is the exact length of the ray through pixel k, averaged over the
 * cell's detector coordinate (arc length for the arc detector; eq. (2)-(3)
 * with the unit-mass blur), with no effective-blur approximation.  Between
 * the rays through the pixel's four corners the chord is smooth, so each
 * piece is integrated by Gauss-Legendre quadrature with quad_points nodes
 * (0 selects 16; at most 24), which reaches FP64 rounding for smooth pieces.
 * FP64 in and out, layouts as fp_forward / fp_back, outputs overwritten;
 * fp_back_reference is the exact adjoint of fp_forward_reference (same
 * entries).  For parallel beams the reference equals the CNSF model
 * (Theorem 1).  Slow by design (thousands of flops per entry): a yardstick
 * for accuracy experiments, not a production path. */
fp_status fp_forward_reference(const fp_geometry *g, const double *image, double *sino,
                               int32_t batch, int32_t quad_points, void *stream);
fp_status fp_back_reference(const fp_geometry *g, const double *sino, double *image,
                            int32_t batch, int32_t quad_points, void *stream);

/* One SIRT step (simultaneous iterative reconstruction; the iterative family
 * the paper targets, Sec. I):
 *     x <- x + relaxation * C .* A^T( R .* (y - A x) ),
 *     R = 1 ./ (A 1),  C = 1 ./ (A^T 1),  1/0 read as 0.
 *   image      device, [batch][ny][nx], the iterate x, updated in place
 *   sino_meas  device, [batch][n_views][n_det], the data y, read only
 *   relaxation lambda, finite (0 < lambda < 2 for convergence)
 *   work       device scratch of batch * n_views * n_det floats, owned by the
 *              caller; holds R .* (y - A x) on return
 * R and C are built on the geometry's device by the first call (one forward
 * and one back projection of ones, then the call waits for them); later
 * calls reuse them.  No clipping is applied to x. */
fp_status fp_sirt_step(const fp_geometry *g, float *image,
                       const float *sino_meas, float relaxation, float *work,
                       int32_t batch, void *stream);

/* The SIRT step of fp_sirt_step for callers that cannot allocate device
 * memory: code under HIP graph capture, serving loops that must not call
 * hipMalloc, harnesses that forbid it.  Arguments, layouts, result and errors
 * are those of fp_sirt_step (the same kernels in the same form, so the same
 * values, wherever that form's scratch fits the array below), with three
 * differences:
 *   - the geometry's SIRT weights must already exist (fp_sirt_prepare or an
 *     earlier fp_sirt_step built them); otherwise FP_ERR_INVALID_ARG;
 *   - the launches' scratch (padded image copies, view-group partial sums)
 *     is a fixed array of FP_NOALLOC_SCRATCH_BYTES in device memory that the
 *     library holds on every device it runs on until the process ends; the
 *     batch is processed in chunks that fit it; where one image's scratch in
 *     fp_sirt_step's form does not fit, the next simpler form whose scratch
 *     fits runs (octant, quarter-turn, plain: equal to FP32 rounding; at
 *     2048 x 2048 the plain form), and a geometry whose single image needs
 *     more than the array in every form gives FP_ERR_UNSUPPORTED (about
 *     2900 x 2900 images and up);
 *   - the call allocates nothing and waits on nothing on the host, and every
 *     call on one device shares that array: calls that can overlap on the
 *     device (different streams, or different host threads without ordering)
 *     race on it and give wrong results.  Order them on one stream. */
#define FP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
fp_status fp_sirt_step_noalloc(const fp_geometry *g, float *image,
                               const float *sino_meas, float relaxation, float *work,
                               int32_t batch, void *stream);

/* Build the SIRT weights R = 1 ./ (A 1) and C = 1 ./ (A^T 1) of a geometry
 * now (fp_sirt_step and fp_sirt_step_multi otherwise build them on first
 * use).  Synchronises `stream` the first time; a no-op afterwards. */
fp_status fp_sirt_prepare(const fp_geometry *g, void *stream);

/* One job of a grouped SIRT step: a geometry and the job's device buffers
 * (batch 1).  Buffers of different jobs must not overlap. */
typedef struct {
    const fp_geometry *geometry;
    float *image;            /* [ny][nx], the iterate, updated in place      */
    const float *sino_meas;  /* [n_views][n_det], the data                   */
    float *work;             /* [n_views][n_det] scratch; R .* (y - A x) on return */
    float relaxation;        /* finite                                        */
} fp_sirt_job;

/* One SIRT step for each of n_jobs jobs whose geometries (image size, views,
 * detector cells, distances) may all differ.  Jobs are grouped by form
 * (quarter-turn or plain) and beam shape, up to 12 per group; per group the
 * padded copies and the forward residuals run as one launch each (every
 * work-group finding its job from the launch's job table), the back
 * projections as one persistent launch whose work-groups drain the (job,
 * tile, view group) items of all jobs in turn, and the updates as one more
 * launch.  (Jobs whose back-projection cell ranges exceed 256 cells per
 * tile run their own back launches.)  This is the execution step of
 * continuous batching: a serving loop admits and retires jobs between calls.
 * The result for each job is that of fp_sirt_step on it alone, to FP32
 * summation order.  All geometries must live on one device.  n_jobs == 0 is
 * a no-op. */
fp_status fp_sirt_step_multi(const fp_sirt_job *jobs, int32_t n_jobs, void *stream);

/* Number of (ray, pixel) pairs with a non-zero entry, counted on the device
 * over the pixels the forward kernel's windows visit, by the footprint's
 * support |s'| < (a + b + tau') / 2 (eq. (18)) in FP32; the result is written
 * to *count on return (the call synchronises `stream`).  Used to price the
 * work of a projection. */
fp_status fp_count_nonzero(const fp_geometry *g, int64_t *count, void *stream);

/* Device scratch bytes one fp_sirt_step call on `batch` images of this
 * geometry takes from the library's reusable per-device buffers (padded
 * image copies and partial sums; the buffers are shared by all calls and
 * kept until the process ends).  0 for NULL or batch < 1.  For admission by
 * free memory. */
size_t fp_sirt_scratch_bytes(const fp_geometry *g, int32_t batch);

/* Device bytes held by the geometry: its tables and, once built, the FP64
 * tables and the SIRT weights.  0 for NULL.  Serving code uses it for admission by free memory. */
size_t fp_geometry_device_bytes(const fp_geometry *g);

/* 1 if the geometry's FP32 projections and SIRT steps run in the
 * quarter-turn form, else 0 (also for NULL).  A square image whose views
 * come in quadruples a quarter turn apart (view v + k n_views/4 at the angle
 * of view v plus k pi/2 for k < 4, to 1e-13 rad; e.g. n_views a multiple of
 * 4 spaced uniformly over 2 pi) is unchanged by a quarter turn of the whole
 * scan, so entry A_{(v + k n_views/4, m), R^k p} equals A_{(v, m), p} with R
 * the quarter turn of the pixel grid (eq. (18) depends only on the ray and
 * the pixel's position relative to it).  That form evaluates each entry once
 * for the four views and applies it to the four quarter-turned images; the
 * results equal the plain form's to FP32 rounding.  The FP64 calls and the
 * reference projector always evaluate every view. */
int32_t fp_geometry_quarter_turn(const fp_geometry *g);

/* Order of the scan symmetry the geometry's FP32 projections and SIRT steps
 * use: 8 (the quarter turns and the reflection across the image diagonal),
 * 4 (the quarter turns only, see fp_geometry_quarter_turn), 1 (none); 0 for
 * NULL.  Order 8 needs a quarter-turn symmetric scan that the reflection
 * across x = y also leaves unchanged: n_views a multiple of 8 and view Q - v
 * at pi/2 minus the angle of view v (Q = n_views / 4; e.g. views
 * 2 pi v / n_views).  The reflection takes the source at angle t to pi/2 - t
 * and detector coordinate s to -s (the cells lie symmetrically about the
 * detector centre), so entry A_{(Q - v, n_det-1-m), D p} equals
 * A_{(v, m), p} with D the reflection of the pixel grid.  With order 8 the
 * back projection of one image (fp_back and the update half of fp_sirt_step
 * with batch 1) evaluates each entry once for eight views (views 0 and Q/2,
 * their own reflections, four); batches of several images, the forward
 * projection and the grouped SIRT step (fp_sirt_step_multi) run in the
 * quarter-turn form.  All forms give the plain form's results to FP32
 * rounding. */
int32_t fp_geometry_symmetry(const fp_geometry *g);

/* Text for the last non-OK status returned on the calling thread ("" if
 * none).  The pointer stays valid until the thread's next fanproj call. */
const char *fp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FANPROJ_H */
