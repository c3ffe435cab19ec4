// Internal declarations shared by the host code (geometry, C ABI) and the
// HIP kernels of libfanproj.  Nothing here is part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
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
constexpr int kFwdMaxUnrolled = 8;   // widest row window with an unrolled variant
// Batch images processed per launch (the kernels are instantiated for
// 1, 2, 4 and 8 images sharing one evaluation of every entry).
constexpr int kMaxBatchChunk = 8;
// Per-ray parameter arrays staged in LDS by the back-projection kernel, in
// addition to one sinogram weight array per image.
constexpr int kBackRayParams = 6;
// Zero-weight cells staged on each side of a tile's cell range, so that a
// pixel's fixed-width window never leaves the staged arrays.
constexpr int kBackPad = 8;
// Widest per-tile window with an unrolled cell loop.
constexpr int kBackMaxUnrolled = 8;
// Cell capacities (per view and tile) the back projection is instantiated for;
// the LDS then holds (kBackRayParams + batch) arrays of that many floats.
constexpr int kBackCaps[] = {64, 128, 256, 512, 1024};
constexpr int kBackMaxCap = 1024;
// LDS the back kernel may use per work-group (two staging buffers).
constexpr size_t kBackLdsLimit = 64 * 1024;
// The back projection splits the views into groups (gridDim.z) until about
// this many work-groups per compute unit are in flight.
constexpr int kBackGroupsPerCu = 8;
constexpr int kBackMaxGroups = 8;

// Read-only description of a geometry as the kernels see it.  All pointers
// are device pointers into one allocation owned by fp_geometry.
struct DevGeom {
    int nx, ny;              // image columns, rows
    int nv, nd;              // views, detector cells
    int tiles_x, tiles_y;    // back-projection tiles
    int max_cells;           // largest per-(view, tile) cell range
    int back_cap;            // LDS capacity (cells) of the back kernel in use
    int back_groups;         // view groups of the back projection (>= 1)
    double pixel;            // delta
    double dsc, dsd;         // source-centre, source-detector distances
    double tau;              // cell width (= pitch)
    double half_diag;        // radius of a disk containing every pixel
    const double2 *views;    // [nv] (cos t, sin t)
    // Per-ray constants, [nv][nd] each (FP32 roundings of FP64 values):
    const float *inv_r;      // 1 / R_m,  R_m = |q(s_m) - p|
    const float *ghr;        // g_m / (2 R_m): half effective blur per unit of R L
    const float *hab;        // (a + b) / 2, a <= b the projected pixel widths
    const float *ia;         // 1 / max(a, tiny)
    const float *nhbia;      // -(b - a) / (2 max(a, tiny))
    const float *ha;         // a / 2
    const float *wb;         // delta^2 / (2 b)
    // [nv][tiles_y * tiles_x]: first cell M0 and count of the cells the tile
    // can touch, the window width T every pixel of the tile evaluates, and
    // (as float bits) the bound H on |s_m - s_k| of its non-zero cells.
    const int4 *tile_cells;
};

enum class FwdMode : int { kPlain = 0, kSirtResidual = 1, kOnes = 2, kCount = 3 };
enum class BackMode : int { kPlain = 0, kSirtUpdate = 1, kOnes = 2 };

// Kernel launchers (projector.hip).  Return the hipError_t of the launch.
// launch_forward: `img` is the caller's [nb][ny][nx] image (unused by the
// kOnes / kCount modes); `work` is device scratch of forward_work_bytes(g, nb)
// bytes for the padded copies.
hipError_t launch_forward(const DevGeom &g, FwdMode mode, int nb, const float *img,
                          float *work, float *out, int *counts, const float *y_meas,
                          const float *row_w, hipStream_t stream);
size_t forward_work_bytes(const DevGeom &g, int nb);
// launch_back: `partial` is device scratch of back_work_bytes(g, nb) bytes
// (may be NULL, which forces a single view group).
hipError_t launch_back(const DevGeom &g, BackMode mode, int nb, const float *sino,
                       float *img, float *partial, const float *col_w, float relaxation,
                       hipStream_t stream);
size_t back_work_bytes(const DevGeom &g, int nb);
// Largest batch chunk the back kernel's LDS holds for this geometry (0 if
// even one image does not fit).
int back_max_batch(const DevGeom &g);

}  // namespace fanproj

struct fp_geometry {
    int device = 0;
    int nx = 0, ny = 0, nv = 0, nd = 0;
    double pixel = 0, dsc = 0, dsd = 0, tau = 0;
    std::vector<double> angles;
    fanproj::DevGeom dev{};
    void *table_block = nullptr;   // one device allocation for all tables
    size_t table_bytes = 0;
    // SIRT weights R = 1/(A 1) and C = 1/(A^T 1), built on first use.
    std::mutex weights_mu;
    bool weights_ready = false;
    float *row_w = nullptr;        // [nv][nd]
    float *col_w = nullptr;        // [ny][nx]
    size_t weight_bytes = 0;
};

namespace fanproj {
// Thread-local error text used by fp_last_error.
void set_error(const std::string &msg);
void clear_error();
fp_status device_error(const char *what, hipError_t e);
}  // namespace fanproj
