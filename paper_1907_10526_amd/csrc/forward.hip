// Forward projection: launchers of the padded image copies and of the
// ray-driven forward kernel (instantiated for FP32 and FP64), and of its
// quarter-turn form for scans with four-fold symmetry (FP32).
#include "kernels.h"

namespace fanproj {
namespace {

// S = 1: the plain walk; S = 4: the quarter-turn walk, G holding the first
// quarter of the views.  Both read the same two padded copies.
template <typename Real, int NB, FwdMode MODE, int S>
hipError_t launch_fwd_t(const DevGeom &g, const Real *img, Real *work, Real *out, int *counts,
                        const Real *y_meas, const Real *row_w, hipStream_t stream) {
    const Real *copies = nullptr;
    if constexpr (MODE == FwdMode::kPlain || MODE == FwdMode::kSirtResidual) {
        const int nrows = std::max(g.nx, g.ny);
        const int width = padded_width(g.nx, g.ny);
        const size_t total = (size_t)NB * nrows * width;
        const unsigned rows_blocks = (unsigned)std::min<size_t>((total + 255) / 256, 4096);
        const int ti = (nrows + 31) / 32, tp = (width + 31) / 32;
        hipLaunchKernelGGL((pad_kernel<Real>), dim3(rows_blocks + (unsigned)(ti * tp * NB)),
                           dim3(32, 8), 0, stream, img, work, g.nx, g.ny, nrows, NB,
                           rows_blocks, ti, tp);
        copies = work;
    }
    // views fastest: consecutive work-groups, which the hardware deals out to
    // the XCDs in turn, take the same ray block of consecutive views, so
    // every XCD gets its share of the long central rays (5 % faster than
    // ray blocks fastest at 512^2 x 720 x 1024)
    constexpr int kRays = fwd_rays_per_block(S);
    dim3 grid(g.nv, (g.nd + kRays - 1) / kRays);
    if (S == 4 && g.fwd_window <= 4) {
        // no window wider than 4 pixels: the instantiation without the
        // unrolled 5- and 6-pixel rows, which needs fewer registers (no
        // spills at 6 waves per SIMD; 3 % faster at 512^2 x 720 x 1024)
        hipLaunchKernelGGL((forward_kernel<Real, NB, MODE, S, 4>), grid, dim3(kFwdThreads), 0,
                           stream, g, copies, out, counts, y_meas, row_w);
    } else {
        hipLaunchKernelGGL((forward_kernel<Real, NB, MODE, S>), grid, dim3(kFwdThreads), 0, stream,
                           g, copies, out, counts, y_meas, row_w);
    }
    return hipGetLastError();
}

template <typename Real, FwdMode MODE>
hipError_t launch_fwd_nb(const DevGeom &g, int nb, const Real *img, Real *work, Real *out,
                         int *counts, const Real *y_meas, const Real *row_w, hipStream_t stream) {
    switch (nb) {
        case 1: return launch_fwd_t<Real, 1, MODE, 1>(g, img, work, out, counts, y_meas, row_w, stream);
        case 2: return launch_fwd_t<Real, 2, MODE, 1>(g, img, work, out, counts, y_meas, row_w, stream);
        case 4: return launch_fwd_t<Real, 4, MODE, 1>(g, img, work, out, counts, y_meas, row_w, stream);
        case 8: return launch_fwd_t<Real, 8, MODE, 1>(g, img, work, out, counts, y_meas, row_w, stream);
        default: return hipErrorInvalidValue;
    }
}

template <FwdMode MODE>
hipError_t launch_fwd_quarter_nb(const DevGeom &g, int nb, const float *img, float *work,
                                 float *out, const float *y_meas, const float *row_w,
                                 hipStream_t stream) {
    switch (nb) {
        case 1: return launch_fwd_t<float, 1, MODE, 4>(g, img, work, out, nullptr, y_meas, row_w, stream);
        case 2: return launch_fwd_t<float, 2, MODE, 4>(g, img, work, out, nullptr, y_meas, row_w, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename Real>
size_t forward_work_bytes(const DevGeom &g, int nb) {
    const size_t nrows = (size_t)std::max(g.nx, g.ny);
    return (size_t)nb * sizeof(Real) * nrows * 2 * (size_t)padded_width(g.nx, g.ny);
}

template <typename Real>
hipError_t launch_forward(const DevGeom &g, FwdMode mode, int nb, const Real *img, Real *work,
                          Real *out, int *counts, const Real *y_meas, const Real *row_w,
                          hipStream_t stream) {
    switch (mode) {
        case FwdMode::kPlain:
            return launch_fwd_nb<Real, FwdMode::kPlain>(g, nb, img, work, out, counts, y_meas,
                                                        row_w, stream);
        case FwdMode::kSirtResidual:
            return launch_fwd_nb<Real, FwdMode::kSirtResidual>(g, nb, img, work, out, counts,
                                                               y_meas, row_w, stream);
        case FwdMode::kOnes:
            return launch_fwd_t<Real, 1, FwdMode::kOnes, 1>(g, img, work, out, counts, y_meas,
                                                            row_w, stream);
        case FwdMode::kCount:
            return launch_fwd_t<Real, 1, FwdMode::kCount, 1>(g, img, work, out, counts, y_meas,
                                                             row_w, stream);
    }
    return hipErrorInvalidValue;
}

namespace {
constexpr int kCountBlocks = 256;
// Sums of n per-ray counts: each of kCountBlocks work-groups sums a stride of
// them into part[blockIdx.x] (integer adds, so the order does not matter);
// count_total_kernel then adds the kCountBlocks sums into *total.
__global__ __launch_bounds__(256) void count_sum_kernel(const int *__restrict__ counts, size_t n,
                                                        unsigned long long *__restrict__ part) {
    __shared__ unsigned long long wsum[256 / 64];
    unsigned long long s = 0;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256)
        s += (unsigned)counts[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(64) void count_total_kernel(const unsigned long long *__restrict__ part,
                                                         unsigned long long *__restrict__ total) {
    unsigned long long s = 0;
    for (int k = threadIdx.x; k < kCountBlocks; k += 64) s += part[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (threadIdx.x == 0) *total = s;
}
}  // namespace

size_t count_work_bytes(const DevGeom &g) {
    return ((size_t)g.nv * g.nd * sizeof(int) + 255) / 256 * 256 +
           (kCountBlocks + 1) * sizeof(unsigned long long);
}

hipError_t launch_count(const DevGeom &g, void *work, hipStream_t stream) {
    int *counts = static_cast<int *>(work);
    auto *part = reinterpret_cast<unsigned long long *>(
        static_cast<char *>(work) + ((size_t)g.nv * g.nd * sizeof(int) + 255) / 256 * 256);
    hipError_t e = launch_forward<float>(g, FwdMode::kCount, 1, nullptr, nullptr, nullptr, counts,
                                         nullptr, nullptr, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_sum_kernel, dim3(kCountBlocks), dim3(256), 0, stream, counts,
                       (size_t)g.nv * g.nd, part);
    hipLaunchKernelGGL(count_total_kernel, dim3(1), dim3(64), 0, stream, part,
                       part + kCountBlocks);
    return hipGetLastError();
}

size_t forward_quarter_work_bytes(const DevGeom &g, int nb) {
    return forward_work_bytes<float>(g, nb);
}

hipError_t launch_forward_quarter(const DevGeom &g, FwdMode mode, int nb, const float *img,
                                  float *work, float *out, const float *y_meas,
                                  const float *row_w, hipStream_t stream) {
    switch (mode) {
        case FwdMode::kPlain:
            return launch_fwd_quarter_nb<FwdMode::kPlain>(g, nb, img, work, out, y_meas, row_w,
                                                          stream);
        case FwdMode::kSirtResidual:
            return launch_fwd_quarter_nb<FwdMode::kSirtResidual>(g, nb, img, work, out, y_meas,
                                                                 row_w, stream);
        default:
            return hipErrorInvalidValue;
    }
}

#define FANPROJ_INSTANTIATE(Real)                                                                  \
    template size_t forward_work_bytes<Real>(const DevGeom &, int);                                \
    template hipError_t launch_forward<Real>(const DevGeom &, FwdMode, int, const Real *, Real *,  \
                                             Real *, int *, const Real *, const Real *,            \
                                             hipStream_t);
FANPROJ_INSTANTIATE(float)
FANPROJ_INSTANTIATE(double)
#undef FANPROJ_INSTANTIATE

}  // namespace fanproj
