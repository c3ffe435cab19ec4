// Internal declarations shared by the host code (geometry, C ABI) and the
// HIP kernels of libfanproj.  Nothing here is part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fanproj.h"

namespace fanproj {

// Back-projection work-group tile: kBackTileW x kBackTileH pixels, 256
// threads, kBackPixPerThread pixels per thread (one column, rows 16 apart).
constexpr int kBackTileW = 16;
constexpr int kBackTileH = 32;
constexpr int kBackThreads = 256;
constexpr int kBackPixPerThread = kBackTileW * kBackTileH / kBackThreads;
// Forward projection: one detector cell (ray) per thread, reading zero-padded
// copies of the image (row-major and transposed) so that the pixels a ray
// visits along a row or column are contiguous and need no bounds checks.
constexpr int kFwdThreads = 256;
constexpr int kFwdPad = 16;          // zero margin on each side of the cross axis
// Row length of both padded copies: the longer image side plus the margins,
// so that every ray sees one row stride and one clamp bound.
__host__ __device__ constexpr int padded_width(int nx, int ny) {
    return (nx > ny ? nx : ny) + 2 * kFwdPad;
}
constexpr int kFwdMaxUnrolled = 8;   // widest row window with an unrolled variant
// A ray marches along the image axis closest to its direction, except that
// a ray whose smaller direction component is at least kFwdAxisShare of the
// larger (within 3 degrees of a diagonal) takes the axis most rays of its
// wave take; its cross axis then still advances s' by at least
// kFwdCrossMin delta per pixel (kFwdAxisShare / sqrt(1 + kFwdAxisShare^2),
// rounded down), against delta / sqrt(2) for the closest axis.
constexpr double kFwdAxisShare = 0.9;
constexpr double kFwdCrossMin = 0.6689;
// Threads per ray of the quarter-turn form's forward: each walks half of the
// ray's row blocks (a work-group then covers kFwdThreads / 2 rays), which,
// compiled for 6 waves per SIMD, made it 6 % faster at 512^2 x 720 x 1024
// (its view count is a quarter of the scan's, so it has few waves).
constexpr int kFwdQuarterParts = 2;
__host__ __device__ constexpr int fwd_rays_per_block(int rotations) {
    return kFwdThreads / (rotations == 4 ? kFwdQuarterParts : 1);
}
// Batch images processed per launch (the kernels are instantiated for
// 1, 2, 4 and 8 images sharing one evaluation of every entry).
constexpr int kMaxBatchChunk = 8;
// Per-ray parameter arrays staged in LDS by the back-projection kernel, in
// addition to one sinogram weight array per image.
constexpr int kBackRayParams = 5;
// Zero-weight cells staged on each side of a tile's cell range, so that a
// pixel's fixed-width window never leaves the staged arrays.
constexpr int kBackPad = 8;
// Widest per-tile window with an unrolled cell loop.
constexpr int kBackMaxUnrolled = 8;
// Values staged per cell by the back projection for a batch chunk of nb
// images: the per-ray parameters and the weights, padded to pairs.
constexpr int back_lds_values(int nb) {
    return kBackRayParams + 1 + 2 * (nb / 2 > 0 ? nb / 2 : 1);
}
// Cell capacities (per view and tile) the back projection is instantiated for;
// the LDS then holds back_lds_values(batch) arrays of that many values.
constexpr int kBackCaps[] = {64, 128, 256, 512, 1024};
constexpr int kBackMaxCap = 1024;
// LDS the back kernel may use per work-group (two staging buffers).
constexpr size_t kBackLdsLimit = 64 * 1024;
// The back projection splits the views into groups (gridDim.z) until about
// this many work-groups per compute unit are in flight.
constexpr int kBackGroupsPerCu = 8;
// Accelerator dies (XCDs) of the part, each with its own L2; the hardware
// hands out work-groups to them round-robin in linear work-group order.
constexpr int kXcds = 8;
constexpr int kBackMaxGroups = 32;

// Per-ray constants, [nv][nd] each, in the kernels' arithmetic type: FP32
// roundings of FP64 values for the production kernels, the FP64 values
// themselves for the FP64 instantiation.
//
// The back projection evaluates an entry in units scaled by the ray's R_m
// (flat detector; 1 for the arc detector and parallel beams), where s' R_m
// and R_m L are its exact numerators: the footprint is homogeneous of degree
// one in (s', hab, a, hc), so the scaled constants below give R_m times the
// same value and no per-entry multiplication by 1 / R_m is needed.
//
// The kRayTables arrays lie `stride` values apart in one block, in the order
// of the accessors below.
template <typename Real>
struct RayTables {
    const Real *base = nullptr;
    size_t stride = 0;
    __host__ __device__ const Real *at(int k) const { return base + (size_t)k * stride; }
    // blur per unit of R L (flat), of L (arc), or tau / 2 (parallel)
    __host__ __device__ const Real *ghr() const { return at(0); }
    // (a + b) / 2, a <= b the projected pixel widths
    __host__ __device__ const Real *hab() const { return at(1); }
    __host__ __device__ const Real *ia() const { return at(2); }     // 1 / max(a, tiny)
    // -(b - a) / (2 max(a, tiny))
    __host__ __device__ const Real *nhbia() const { return at(3); }
    __host__ __device__ const Real *ha() const { return at(4); }     // a / 2
    __host__ __device__ const Real *wb() const { return at(5); }     // delta^2 / (2 b)
    __host__ __device__ const Real *bgh() const { return at(6); }    // ghr R_m
    __host__ __device__ const Real *bhab() const { return at(7); }   // hab R_m
    __host__ __device__ const Real *bia() const { return at(8); }    // ia / R_m
    __host__ __device__ const Real *bha() const { return at(9); }    // ha R_m
    // wb / bgh: the back projection divides an entry's footprint by R_m L
    // alone and folds the blur constant into the staged weight
    __host__ __device__ const Real *bwg() const { return at(10); }
};
constexpr int kRayTables = 11;

// Read-only description of a geometry as the kernels see it.  All pointers
// are device pointers owned by fp_geometry.
struct DevGeom {
    int nx, ny;              // image columns, rows
    int nv, nd;              // views, detector cells
    int tiles_x, tiles_y;    // back-projection tiles
    int max_cells;           // largest per-(view, tile) cell range
    int back_cap;            // LDS capacity (cells) of the back kernel in use
    int back_groups;         // view groups of the back projection (>= 1)
    // Octant form only (nv = quarter_views / 2 + 1 base views of a scan of
    // 4 quarter_views views): views per quarter turn; 0 in the other forms.
    int quarter_views;
    // Upper bound on the forward walk's window width in pixels (a launch
    // heuristic: a wider window is still walked correctly, by the loop).
    int fwd_window;
    int beam;                // FP_FAN_FLAT, FP_FAN_ARC or FP_PARALLEL
    double pixel;            // delta
    double dsc, dsd;         // source-centre, source-detector distances
    double tau;              // cell width (aperture)
    double pitch;            // distance between cell centres
    // Cell spacing in the coordinate the back projection places windows in:
    // the pitch (flat: detector coordinate; parallel: e.x), or the angle
    // pitch / D_sd (arc).
    double cell_step;
    double half_diag;        // radius of a disk containing every pixel
    const double2 *views;    // [nv] (cos t, sin t)
    // arc detector only: (cos g_m, sin g_m), g_m = s_m / D_sd, for cells
    // m = -kBackPad .. nd + kBackPad - 1 at index m + kBackPad; and
    // (cos, sin) of t * (pitch / D_sd) for t < kBackMaxUnrolled
    const double2 *arc_cells;
    const float2 *arc_rot;
    const double2 *arc_rot64;
    RayTables<float> r32;
    RayTables<double> r64;   // built on the first FP64 call
    // [nv][tiles_y * tiles_x]: first cell M0 and count of the cells the tile
    // can touch, the window width T every pixel of the tile evaluates, and
    // (as float bits) the bound H on |s_m - s_k| of its non-zero cells.
    const int4 *tile_cells;
};

template <typename Real>
__host__ __device__ inline const RayTables<Real> &ray_tables(const DevGeom &g);
// The arc rotations in the kernels' arithmetic type, as (cos, sin) pairs.
template <typename Real>
__device__ inline void arc_rotation(const DevGeom &g, int t, Real &c, Real &s);
template <>
__device__ inline void arc_rotation<float>(const DevGeom &g, int t, float &c, float &s) {
    const float2 r = g.arc_rot[t];
    c = r.x;
    s = r.y;
}
template <>
__device__ inline void arc_rotation<double>(const DevGeom &g, int t, double &c, double &s) {
    const double2 r = g.arc_rot64[t];
    c = r.x;
    s = r.y;
}
template <>
__host__ __device__ inline const RayTables<float> &ray_tables<float>(const DevGeom &g) {
    return g.r32;
}
template <>
__host__ __device__ inline const RayTables<double> &ray_tables<double>(const DevGeom &g) {
    return g.r64;
}

enum class FwdMode : int { kPlain = 0, kSirtResidual = 1, kOnes = 2, kCount = 3 };
enum class BackMode : int { kPlain = 0, kSirtUpdate = 1, kOnes = 2 };

// Kernel launchers (forward.hip, back*.hip / back.cpp), instantiated for
// Real = float and double.
// Return the hipError_t of the launch.
// launch_forward: `img` is the caller's [nb][ny][nx] image (unused by the
// kOnes / kCount modes); `work` is device scratch of forward_work_bytes
// bytes for the padded copies.
template <typename Real>
hipError_t launch_forward(const DevGeom &g, FwdMode mode, int nb, const Real *img, Real *work,
                          Real *out, int *counts, const Real *y_meas, const Real *row_w,
                          hipStream_t stream);
template <typename Real>
size_t forward_work_bytes(const DevGeom &g, int nb);
// launch_back: `partial` is device scratch of back_work_bytes bytes (may be
// NULL, which forces a single view group).
template <typename Real>
hipError_t launch_back(const DevGeom &g, BackMode mode, int nb, const Real *sino, Real *img,
                       Real *partial, const Real *col_w, Real relaxation, hipStream_t stream);
template <typename Real>
size_t back_work_bytes(const DevGeom &g, int nb);
// launch_back for one beam shape (BEAM = FP_FAN_FLAT, FP_FAN_ARC or
// FP_PARALLEL); launch_back dispatches on g.beam.
template <typename Real, int BEAM>
hipError_t launch_back_beam(const DevGeom &g, BackMode mode, int nb, const Real *sino, Real *img,
                            Real *partial, const Real *col_w, Real relaxation, hipStream_t stream);
// Largest batch chunk the back kernel's LDS holds for this geometry (0 if
// even one image does not fit).
template <typename Real>
int back_max_batch(const DevGeom &g);

// Number of non-zero entries (fp_count_nonzero): the forward's count mode
// into `work` (count_work_bytes(g) bytes), then a two-level sum, left as an
// unsigned 64-bit integer in the last 8 bytes of `work`.
size_t count_work_bytes(const DevGeom &g);
hipError_t launch_count(const DevGeom &g, void *work, hipStream_t stream);

// Quarter-turn forms (FP32) for a square image whose views come in
// quadruples a quarter turn apart (view v + k nv at angle t_v + k pi/2, nv a
// quarter of the views, k < 4): g describes the first quarter of the views,
// the tables of which are a prefix of the full geometry's.  The entries of
// view v + k nv on an image equal those of view v on the image turned by k
// quarter turns, so each entry is evaluated once for four views.  Sinograms
// keep their full [nb][4 nv][nd] layout; at most kQuarterMaxChunk images per
// launch.  launch_forward_quarter: modes kPlain and kSirtResidual (row_w the
// full view set's), `work` of forward_quarter_work_bytes(g, nb) bytes for
// four padded copies per image.  launch_back_quarter: modes kPlain and
// kSirtUpdate, `partial` of back_quarter_work_bytes(g, nb) bytes.
constexpr int kQuarterMaxChunk = 2;
size_t forward_quarter_work_bytes(const DevGeom &g, int nb);
hipError_t launch_forward_quarter(const DevGeom &g, FwdMode mode, int nb, const float *img,
                                  float *work, float *out, const float *y_meas,
                                  const float *row_w, hipStream_t stream);
size_t back_quarter_work_bytes(const DevGeom &g, int nb);
hipError_t launch_back_quarter(const DevGeom &g, BackMode mode, int nb, const float *sino,
                               float *img, float *partial, const float *col_w, float relaxation,
                               hipStream_t stream);
template <int BEAM>
hipError_t launch_back_quarter_beam(const DevGeom &g, BackMode mode, int nb, const float *sino,
                                    float *img, float *partial, const float *col_w,
                                    float relaxation, hipStream_t stream);

// Octant form of the back projection (FP32, one image per launch) for a
// quarter-turn symmetric scan that is also unchanged by the reflection
// across the image diagonal x = y: views t_v and t_{Q-v} with
// t_v + t_{Q-v} = pi/2 (Q = nv_scan / 4; then nv_scan % 8 == 0) and cells
// symmetric about the detector centre.  The reflection D(i, j) = (j, i)
// takes ray (v, m) to ray (Q - v, nd-1-m), so with the quarter turns the
// entry A_{(v,m),p} also equals A_{((Q - v + k Q) mod 4Q, nd-1-m), R^k D p}:
// each entry is evaluated once for eight views.  g describes the base views
// 0 .. Q/2 (a prefix of the full tables, quarter_views = Q); views 0 and
// Q/2 are their own reflections and serve four views.  Modes kPlain and
// kSirtUpdate, `partial` of back_octant_work_bytes(g) bytes.  (The forward
// projection of such a scan runs in the quarter-turn form: its ray walk
// reads one pixel value per non-zero entry in either form, and an eight-view
// walk, with twice the reads and accumulators per evaluated entry, measured
// slower.)
size_t back_octant_work_bytes(const DevGeom &g);
hipError_t launch_back_octant(const DevGeom &g, BackMode mode, const float *sino, float *img,
                              float *partial, const float *col_w, float relaxation,
                              hipStream_t stream);
template <int BEAM>
hipError_t launch_back_octant_beam(const DevGeom &g, BackMode mode, const float *sino,
                                   float *img, float *partial, const float *col_w,
                                   float relaxation, hipStream_t stream);

// The form a single-geometry SIRT step runs in: every view on its own, the
// quarter-turn form (four views per evaluated entry), or the quarter-turn
// forward with the octant back projection (eight views per evaluated entry
// of the back projection).
enum class Form : int { kPlain = 0, kQuarter = 1, kOctant = 2 };

// Grouped SIRT step: several jobs, each with its own geometry; one launch
// for the padded copies and one for the forward residuals of all of them,
// then each job's back update.  Up to kMaxJobsPerLaunch job descriptors
// travel in the kernel arguments.
constexpr int kMaxJobsPerLaunch = 12;
struct MultiJob {
    DevGeom g;
    const float *image;     // [ny][nx] iterate, read by the forward phase
    float *copies;          // the interleaved padded copies (scratch)
    float *image_out;       // the iterate, updated by the back phase
    const float *y_meas;    // [nv][nd]
    float *work;            // [nv][nd] residual R .* (y - A x)
    const float *row_w, *col_w;
    float relaxation;
    unsigned fwd_begin;     // first forward work-group of this job
    unsigned back_begin;    // first back-projection item (tile, view group) of this job
    float *partial;         // view-group partials of the back update (scratch)
};
struct MultiArgs {
    int n;
    // 1: every job in the quarter-turn form (g = the geometry's dev_quarter);
    // 0: every job in the plain form
    int quarter;
    int beam;               // the beam shape of every job
    int cap;                // the largest back_cap of the jobs
    unsigned fwd_blocks;
    unsigned back_items;    // back-projection items of all jobs
    MultiJob job[kMaxJobsPerLaunch];
};
static_assert(sizeof(MultiArgs) <= 4000, "kernel arguments must stay under 4 KB");
// Scratch of one job of a grouped step (copies, partials).
size_t multi_copies_bytes(const DevGeom &g);
size_t multi_partial_bytes(const DevGeom &g, bool quarter);
// Largest back-projection LDS capacity the grouped back phase takes; jobs
// with larger cell ranges run their own back launches.
constexpr int kMultiMaxCap = 256;
// Launch the phases for args.job[0 .. n) (multi.hip): the padded copies and
// the forward residuals of all jobs (one launch each), the back
// projections of all jobs as one persistent launch draining (job, tile,
// view group) items, and one launch finishing all their updates.
// copies/partial/fwd_begin/back_begin must be filled in, each job's buffers
// of multi_copies_bytes and multi_partial_bytes bytes.
hipError_t launch_sirt_multi(const MultiArgs &args, hipStream_t stream);

// A point recorded on a stream after one call's launches (one event per
// call, abi.cpp): the call's scratch buffer and its geometries keep it, and
// whoever needs that work finished (the buffer's next user on another
// stream, the memory of a destroyed geometry) waits for it.  The events are
// created without the system-scope fence (they order work on the device and
// tell the host that work has finished; nothing reads the results through
// them) and go back to a per-device free list when the last holder lets go.
struct Mark {
    hipEvent_t ev = nullptr;
    int dev = 0;
    ~Mark();
};
using MarkPtr = std::shared_ptr<Mark>;
// Records a mark on `s` (device `dev` current); nullptr if that fails.
MarkPtr record_mark(int dev, hipStream_t s);

}  // namespace fanproj

struct fp_geometry {
    int device = 0;
    int nx = 0, ny = 0, nv = 0, nd = 0, beam = FP_FAN_FLAT;
    double pixel = 0, dsc = 0, dsd = 0, tau = 0, pitch = 0;
    std::vector<double> angles;
    fanproj::DevGeom dev{};
    // Quarter-turn symmetry (nx == ny, views in quarter-turn quadruples):
    // dev_quarter is dev restricted to the first quarter of the views (same
    // tables, nv / 4 views, its own view-group count); FP32 projections and
    // SIRT steps then run in the quarter-turn form.
    bool quarter = false;
    fanproj::DevGeom dev_quarter{};
    // Octant symmetry (quarter-turn symmetric and unchanged by the reflection
    // across the diagonal): dev_octant is dev restricted to the views
    // 0 .. nv / 8 with quarter_views = nv / 4; single-image FP32 back
    // projections (and the back half of single-image SIRT steps) then run in
    // the octant form.
    bool octant = false;
    fanproj::DevGeom dev_octant{};
    void *table_block = nullptr;   // one device allocation for the FP32 tables
    size_t table_bytes = 0, table_cap = 0;   // bytes used, bytes of the block
    // FP64 per-ray tables, built on the first FP64 call.
    std::mutex f64_mu;
    bool f64_ready = false;
    void *f64_block = nullptr;
    size_t f64_bytes = 0, f64_cap = 0;
    // SIRT weights R = 1/(A 1) and C = 1/(A^T 1), built on first use.
    std::mutex weights_mu;
    bool weights_ready = false;
    float *row_w = nullptr;        // [nv][nd]
    float *col_w = nullptr;        // [ny][nx]
    size_t weight_bytes = 0, row_cap = 0, col_cap = 0;
    // The streams that launched work on the geometry, each with the mark
    // recorded after its latest launches: the memory of a destroyed geometry
    // is reused only after these (not after the whole device).  untracked: a
    // mark could not be recorded, so destroy waits for the device.
    std::mutex use_mu;
    std::vector<std::pair<hipStream_t, fanproj::MarkPtr>> uses;
    bool untracked = false;
};

namespace fanproj {
// Makes the geometry's device current for the duration of a call and
// restores the caller's device afterwards.
class DeviceGuard {
  public:
    explicit DeviceGuard(int dev) {
        err_ = hipGetDevice(&prev_);
        if (err_ == hipSuccess && prev_ != dev) {
            err_ = hipSetDevice(dev);
            switched_ = err_ == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (switched_) (void)hipSetDevice(prev_);
    }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
    hipError_t status() const { return err_; }

  private:
    int prev_ = 0;
    bool switched_ = false;
    hipError_t err_ = hipSuccess;
};

// The parts of the SIRT step shared by the SIRT entry points (abi.cpp).
// sirt_check: the argument checks of fp_sirt_step (geometry, batch,
// relaxation, device pointers).  sirt_form: the form a step of `batch`
// images runs in (the octant form for one image where the geometry has it;
// else the quarter-turn form where the geometry has it; else the plain
// one); `form` below must be one the geometry has.  sirt_max_chunk: the
// largest batch chunk one launch pair takes.  sirt_scratch_bytes: device
// scratch one step needs for chunks of nb images (padded copies, then
// view-group partials at *partial_offset).  sirt_step_launch: the launches,
// in chunks of at most max_nb images, with `scratch` of
// sirt_scratch_bytes(g, max_nb, form) bytes; the weights must have been
// built.
fp_status sirt_check(const fp_geometry *g, const float *image, const float *sino_meas,
                     float relaxation, const float *work, int32_t batch, const char *fn);
Form sirt_form(const fp_geometry *g, int32_t batch);
int sirt_max_chunk(const fp_geometry *g, Form form);
size_t sirt_scratch_bytes(const fp_geometry *g, int nb, Form form, size_t *partial_offset);
fp_status sirt_step_launch(const fp_geometry *g, float *image, const float *sino_meas,
                           float relaxation, float *work, int32_t batch, int max_nb, Form form,
                           void *scratch, hipStream_t s, const char *fn);

// The reference projector (reference.hip): forward (true) or its adjoint
// over `batch` images, FP64, `quad` Gauss-Legendre points per smooth piece.
hipError_t launch_reference(const fp_geometry *g, bool forward, const double *in, double *out,
                            int batch, int quad, hipStream_t s);
// Uploads the FP64 per-ray tables if they are not there yet (thread-safe).
fp_status ensure_f64_tables(fp_geometry *g);
// Device memory of geometries (pool.cpp): pool_alloc takes an idle block of
// a destroyed geometry that fits (waiting for the work queued with it) or
// allocates one; *capacity receives the block's size, which pool_release
// needs.  pool_release hands blocks back with the marks of the work still
// queued against them; it does not wait.  Device `dev` must be current for
// both.
hipError_t pool_alloc(int dev, size_t bytes, void **out, size_t *capacity);
void pool_release(int dev, const std::vector<std::pair<void *, size_t>> &blocks,
                  const std::vector<MarkPtr> &after);
// Keeps `m`, recorded after the work just queued on `s` for the geometry, as
// that stream's latest use of it (a null mark makes destroy wait for the
// device).
void note_use(const fp_geometry *g, hipStream_t s, const MarkPtr &m);
// Thread-local error text used by fp_last_error.
void set_error(const std::string &msg);
void clear_error();
fp_status device_error(const char *what, hipError_t e);
}  // namespace fanproj
