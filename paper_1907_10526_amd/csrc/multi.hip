// Grouped SIRT step of several jobs with different geometries: one launch
// for the padded copies and one for the forward residuals of all jobs, one
// persistent launch for the back projections of all jobs and one for their
// updates.
#include "kernels.h"

namespace fanproj {
namespace {

// ---------------------------------------------------------------------------
// Grouped SIRT step over several jobs: work-group b of a phase belongs to the
// last job whose first work-group is <= b (jobs are in order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int multi_job_of(const MultiArgs &A, unsigned b) {
    int j = 0;
    for (int k = 1; k < A.n; ++k)
        if (A.job[k].fwd_begin <= b) j = k;
    return j;
}

// Padded copies of every job's iterate: blockIdx.y = job; the blocks of a
// job stride over its row copy and over the 32 x 32 tiles of its column copy.
__global__ __launch_bounds__(256) void pad_multi_kernel(const MultiArgs A) {
    __shared__ float tile[32][33];
    const MultiJob &J = A.job[blockIdx.y];
    const int nx = J.g.nx, ny = J.g.ny, nrows = max(nx, ny);
    const int tid = threadIdx.y * 32 + threadIdx.x;
    pad_rows_body<float>(J.image, J.copies, nx, ny, nrows, 1, (size_t)blockIdx.x * 256 + tid,
                         (size_t)gridDim.x * 256);
    const int w = padded_width(nx, ny);
    const int ti = (nrows + 31) / 32, tp = (w + 31) / 32;
    for (int t = blockIdx.x; t < ti * tp; t += gridDim.x)
        pad_cols_tile<float>(J.image, J.copies + w, nx, ny, nrows, (t % ti) * 32, (t / ti) * 32,
                             tile);
}

// The forward residuals of every job; R = 1 (plain) or 4 (quarter-turn form:
// the forward walk's rotations, see forward_block).
template <int R>
__global__ __launch_bounds__(kFwdThreads, R == 1 ? 8 : 6) void forward_multi_kernel(
    const MultiArgs A) {
    const int j = multi_job_of(A, blockIdx.x);
    const MultiJob &J = A.job[j];
    const unsigned local = blockIdx.x - J.fwd_begin;
    // (views fastest, as in the single-job launch)
    const unsigned nv = (unsigned)J.g.nv;
    forward_block<float, 1, FwdMode::kSirtResidual, R>(J.g, local % nv, local / nv, J.copies,
                                                      J.work, nullptr, J.y_meas, J.row_w);
}

// The back projections of every job: a persistent grid whose work-groups
// take (job, tile, view group) items in turn, item k by work-group
// k mod gridDim.x, each writing its view group's sums to the job's partials
// (NB = 4 for the quarter-turn form, whose four images are the four view
// quarters; 1 for the plain form).  Items are whole tiles, so every pixel's
// sum is formed by one work-group, as in the single-job kernel.
template <int NB, int CAP, int BEAM>
__global__ __launch_bounds__(kBackThreads, min_waves(NB, sizeof(float))) void back_multi_kernel(
    const MultiArgs A) {
    __shared__ BackLds<float, NB, CAP> lds[2];
    for (unsigned item = blockIdx.x; item < A.back_items; item += gridDim.x) {
        int j = 0;
        for (int k = 1; k < A.n; ++k)
            if (A.job[k].back_begin <= item) j = k;
        const MultiJob &J = A.job[j];
        const unsigned local = item - J.back_begin;
        const unsigned ntiles = (unsigned)(J.g.tiles_x * J.g.tiles_y);
        const int tile = (int)(local % ntiles), group = (int)(local / ntiles);
        back_block<float, NB, CAP, BackMode::kPlain, BEAM>(
            lds, J.g, tile % J.g.tiles_x, tile / J.g.tiles_x, group, J.g.back_groups, true, J.work,
            nullptr, J.partial, nullptr, 0.0f);
    }
}

// Every job's update x += lambda C .* (sum of its partials): blockIdx.z =
// job; quarter-turn form: 32 x 32 tiles combining the four rotations
// (finalize_quarter_tile); plain form: a block stride over the pixels.
__global__ __launch_bounds__(1024) void finalize_quarter_multi_kernel(const MultiArgs A) {
    const MultiJob &J = A.job[blockIdx.z];
    const int n = J.g.nx, i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    if (i0 >= n || j0 >= n) return;   // (uniform over the block)
    finalize_quarter_tile<BackMode::kSirtUpdate>(J.partial, J.g.back_groups, 4, n, 0, i0, j0,
                                                 J.image_out, J.col_w, J.relaxation);
}

__global__ __launch_bounds__(256) void finalize_plain_multi_kernel(const MultiArgs A) {
    const MultiJob &J = A.job[blockIdx.z];
    const size_t npix = (size_t)J.g.nx * J.g.ny;
    const int groups = J.g.back_groups;
    for (size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x; pix < npix;
         pix += (size_t)gridDim.x * 256) {
        float z = 0.0f;
        for (int g = 0; g < groups; ++g) z += J.partial[(size_t)g * npix + pix];
        J.image_out[pix] += J.relaxation * J.col_w[pix] * z;
    }
}

template <int NB, int BEAM>
hipError_t launch_back_multi_cap(const MultiArgs &A, unsigned grid, hipStream_t stream) {
    switch (A.cap) {
        case 64:
            hipLaunchKernelGGL((back_multi_kernel<NB, 64, BEAM>), dim3(grid), dim3(kBackThreads), 0,
                               stream, A);
            return hipGetLastError();
        case 128:
            hipLaunchKernelGGL((back_multi_kernel<NB, 128, BEAM>), dim3(grid), dim3(kBackThreads),
                               0, stream, A);
            return hipGetLastError();
        case 256:
            hipLaunchKernelGGL((back_multi_kernel<NB, 256, BEAM>), dim3(grid), dim3(kBackThreads),
                               0, stream, A);
            return hipGetLastError();
        default:
            return hipErrorInvalidValue;
    }
}

template <int NB>
hipError_t launch_back_multi(const MultiArgs &A, unsigned grid, hipStream_t stream) {
    switch (A.beam) {
        case FP_FAN_FLAT: return launch_back_multi_cap<NB, FP_FAN_FLAT>(A, grid, stream);
        case FP_FAN_ARC: return launch_back_multi_cap<NB, FP_FAN_ARC>(A, grid, stream);
        case FP_PARALLEL: return launch_back_multi_cap<NB, FP_PARALLEL>(A, grid, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t multi_copies_bytes(const DevGeom &g) { return forward_work_bytes<float>(g, 1); }

size_t multi_partial_bytes(const DevGeom &g, bool quarter) {
    return (size_t)g.back_groups * (quarter ? 4 : 1) * g.nx * g.ny * sizeof(float);
}

hipError_t launch_sirt_multi(const MultiArgs &A, hipStream_t stream) {
    if (A.n < 1) return hipSuccess;
    if (A.quarter) {
        hipLaunchKernelGGL(pad_multi_kernel, dim3(64, A.n), dim3(32, 8), 0, stream, A);
        hipLaunchKernelGGL(forward_multi_kernel<4>, dim3(A.fwd_blocks), dim3(kFwdThreads), 0,
                           stream, A);
    } else {
        hipLaunchKernelGGL(pad_multi_kernel, dim3(64, A.n), dim3(32, 8), 0, stream, A);
        hipLaunchKernelGGL(forward_multi_kernel<1>, dim3(A.fwd_blocks), dim3(kFwdThreads), 0,
                           stream, A);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (A.cap > kMultiMaxCap) {
        // wide cell ranges: each job's own back launch
        for (int k = 0; k < A.n && e == hipSuccess; ++k) {
            const MultiJob &J = A.job[k];
            e = A.quarter ? launch_back_quarter(J.g, BackMode::kSirtUpdate, 1, J.work,
                                                J.image_out, J.partial, J.col_w, J.relaxation,
                                                stream)
                          : launch_back<float>(J.g, BackMode::kSirtUpdate, 1, J.work,
                                               J.image_out, J.partial, J.col_w, J.relaxation,
                                               stream);
        }
        return e;
    }
    // a resident grid (about the work-groups the chip holds at once)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1) {
        (void)hipGetLastError();
        cus = 256;
    }
    const unsigned grid = std::min<unsigned>(A.back_items, (unsigned)(kBackGroupsPerCu * cus));
    e = A.quarter ? launch_back_multi<4>(A, grid, stream) : launch_back_multi<1>(A, grid, stream);
    if (e != hipSuccess) return e;
    int nmax = 0;
    for (int k = 0; k < A.n; ++k) nmax = std::max(nmax, std::max(A.job[k].g.nx, A.job[k].g.ny));
    if (A.quarter) {
        const unsigned t = (unsigned)((nmax + 31) / 32);
        hipLaunchKernelGGL(finalize_quarter_multi_kernel, dim3(t, t, A.n), dim3(32, 32), 0, stream,
                           A);
    } else {
        const unsigned blocks = (unsigned)std::min<size_t>(((size_t)nmax * nmax + 255) / 256, 1024);
        hipLaunchKernelGGL(finalize_plain_multi_kernel, dim3(blocks, 1, A.n), dim3(256), 0, stream,
                           A);
    }
    return hipGetLastError();
}

}  // namespace fanproj
