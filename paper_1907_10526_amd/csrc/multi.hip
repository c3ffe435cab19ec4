// Grouped SIRT step of several jobs with different geometries: one launch
// for the padded copies and one for the forward residuals of all jobs, then
// each job's back update (which splits its views over work-group groups).
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
// job stride over its row copies and over the 32 x 32 tiles of its column
// copies.  S: copy slots per row (2 plain, 4 quarter-turn form).
template <int S>
__global__ __launch_bounds__(256) void pad_multi_kernel(const MultiArgs A) {
    __shared__ float tile[32][33];
    const MultiJob &J = A.job[blockIdx.y];
    const int nx = J.g.nx, ny = J.g.ny, nrows = max(nx, ny);
    const int tid = threadIdx.y * 32 + threadIdx.x;
    pad_rows_body<float, S>(J.image, J.copies, nx, ny, nrows, 1, (size_t)blockIdx.x * 256 + tid,
                            (size_t)gridDim.x * 256);
    const int w = padded_width(nx, ny);
    const int ti = (nrows + 31) / 32, tp = (w + 31) / 32;
    for (int t = blockIdx.x; t < ti * tp; t += gridDim.x)
        pad_cols_tile<float, S>(J.image, J.copies + w, nx, ny, nrows, (t % ti) * 32,
                                (t / ti) * 32, tile);
}

// The forward residuals of every job; R = 1 (plain) or 4 (quarter-turn form:
// the forward walk's rotations, see forward_block).
template <int R>
__global__ __launch_bounds__(kFwdThreads, R == 1 ? 8 : 1) void forward_multi_kernel(
    const MultiArgs A) {
    const int j = multi_job_of(A, blockIdx.x);
    const MultiJob &J = A.job[j];
    const unsigned local = blockIdx.x - J.fwd_begin;
    const unsigned bx = (J.g.nd + kFwdThreads - 1) / kFwdThreads;
    forward_block<float, 1, FwdMode::kSirtResidual, R>(J.g, local / bx, local % bx, J.copies,
                                                      J.work, nullptr, J.y_meas, J.row_w);
}

}  // namespace

hipError_t launch_sirt_multi(const MultiArgs &A, hipStream_t stream) {
    if (A.n < 1) return hipSuccess;
    if (A.quarter) {
        hipLaunchKernelGGL(pad_multi_kernel<4>, dim3(64, A.n), dim3(32, 8), 0, stream, A);
        hipLaunchKernelGGL(forward_multi_kernel<4>, dim3(A.fwd_blocks), dim3(kFwdThreads), 0,
                           stream, A);
    } else {
        hipLaunchKernelGGL(pad_multi_kernel<2>, dim3(64, A.n), dim3(32, 8), 0, stream, A);
        hipLaunchKernelGGL(forward_multi_kernel<1>, dim3(A.fwd_blocks), dim3(kFwdThreads), 0,
                           stream, A);
    }
    hipError_t e = hipGetLastError();
    // The back projection of a small job alone still fills the device with
    // its view groups; a grouped back kernel, one work-group per tile and
    // job, measured slower.
    for (int k = 0; k < A.n && e == hipSuccess; ++k) {
        const MultiJob &J = A.job[k];
        e = A.quarter ? launch_back_quarter(J.g, BackMode::kSirtUpdate, 1, J.work, J.image_out,
                                            J.partial, J.col_w, J.relaxation, stream)
                      : launch_back<float>(J.g, BackMode::kSirtUpdate, 1, J.work, J.image_out,
                                           J.partial, J.col_w, J.relaxation, stream);
    }
    return e;
}

}  // namespace fanproj
