// Grouped SIRT step: the three phases (padded copies, forward residual, back
// update) of several jobs with different geometries, one launch per phase.
#include "kernels.h"

namespace fanproj {
namespace {

// ---------------------------------------------------------------------------
// Grouped SIRT step over several jobs: work-group b of a phase belongs to the
// last job whose first work-group is <= b (jobs are in order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int multi_job_of(const MultiArgs &A, unsigned b, bool back) {
    int j = 0;
    for (int k = 1; k < A.n; ++k)
        if ((back ? A.job[k].back_begin : A.job[k].fwd_begin) <= b) j = k;
    return j;
}

// Padded copies of every job's iterate: blockIdx.y = job; the blocks of a
// job stride over its row copy and over the 32 x 32 tiles of its column copy.
__global__ __launch_bounds__(256) void pad_multi_kernel(const MultiArgs A) {
    __shared__ float tile[32][33];
    const MultiJob &J = A.job[blockIdx.y];
    const int nx = J.g.nx, ny = J.g.ny, nrows = max(nx, ny);
    const int tid = threadIdx.y * 32 + threadIdx.x;
    pad_rows_body<float>(J.image, J.rows, nx, ny, nrows, 1, (size_t)blockIdx.x * 256 + tid,
                         (size_t)gridDim.x * 256);
    const int ti = (nrows + 31) / 32, tp = (ny + 2 * kFwdPad + 31) / 32;
    for (int t = blockIdx.x; t < ti * tp; t += gridDim.x)
        pad_cols_tile<float>(J.image, J.cols, nx, ny, nrows, (t % ti) * 32, (t / ti) * 32, tile);
}

__global__ __launch_bounds__(kFwdThreads) void forward_multi_kernel(const MultiArgs A) {
    const int j = multi_job_of(A, blockIdx.x, false);
    const MultiJob &J = A.job[j];
    const unsigned local = blockIdx.x - J.fwd_begin;
    const unsigned bx = (J.g.nd + kFwdThreads - 1) / kFwdThreads;
    forward_block<float, 1, FwdMode::kSirtResidual>(J.g, local / bx, local % bx, J.rows, J.cols,
                                                   J.work, nullptr, J.y_meas, J.row_w);
}

template <int CAP>
__global__ __launch_bounds__(kBackThreads) void back_multi_kernel(const MultiArgs A) {
    const int j = multi_job_of(A, blockIdx.x, true);
    const MultiJob &J = A.job[j];
    const unsigned local = blockIdx.x - J.back_begin;
    const int tx = local % J.g.tiles_x, ty = local / J.g.tiles_x;
    __shared__ BackLds<float, 1, CAP> lds[2];
    switch (J.g.beam) {
        case FP_FAN_ARC:
            back_block<float, 1, CAP, BackMode::kSirtUpdate, FP_FAN_ARC>(
                lds, J.g, tx, ty, 0, 1, J.work, J.image_out, nullptr, J.col_w, J.relaxation);
            break;
        case FP_PARALLEL:
            back_block<float, 1, CAP, BackMode::kSirtUpdate, FP_PARALLEL>(
                lds, J.g, tx, ty, 0, 1, J.work, J.image_out, nullptr, J.col_w, J.relaxation);
            break;
        default:
            back_block<float, 1, CAP, BackMode::kSirtUpdate, FP_FAN_FLAT>(
                lds, J.g, tx, ty, 0, 1, J.work, J.image_out, nullptr, J.col_w, J.relaxation);
            break;
    }
}

}  // namespace

hipError_t launch_sirt_multi(const MultiArgs &A, hipStream_t stream) {
    if (A.n < 1) return hipSuccess;
    int cap = 0;
    for (int k = 0; k < A.n; ++k) cap = std::max(cap, A.job[k].g.back_cap);
    hipLaunchKernelGGL(pad_multi_kernel, dim3(64, A.n), dim3(32, 8), 0, stream, A);
    hipLaunchKernelGGL(forward_multi_kernel, dim3(A.fwd_blocks), dim3(kFwdThreads), 0, stream, A);
    switch (cap) {
        case 64: hipLaunchKernelGGL(back_multi_kernel<64>, dim3(A.back_blocks), dim3(kBackThreads), 0, stream, A); break;
        case 128: hipLaunchKernelGGL(back_multi_kernel<128>, dim3(A.back_blocks), dim3(kBackThreads), 0, stream, A); break;
        case 256: hipLaunchKernelGGL(back_multi_kernel<256>, dim3(A.back_blocks), dim3(kBackThreads), 0, stream, A); break;
        case 512: hipLaunchKernelGGL(back_multi_kernel<512>, dim3(A.back_blocks), dim3(kBackThreads), 0, stream, A); break;
        case 1024: hipLaunchKernelGGL(back_multi_kernel<1024>, dim3(A.back_blocks), dim3(kBackThreads), 0, stream, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fanproj
