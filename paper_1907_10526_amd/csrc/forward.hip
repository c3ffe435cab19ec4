// Forward projection: launchers of the padded image copies and of the
// ray-driven forward kernel (instantiated for FP32 and FP64), and of its
// quarter-turn form for scans with four-fold symmetry (FP32).
#include "kernels.h"

namespace fanproj {
namespace {

// S = 1: the plain walk over copies of 2 slots; S = 4: the
// quarter-turn walk over 4 slots, G holding the first quarter of the views.
template <typename Real, int NB, FwdMode MODE, int S>
hipError_t launch_fwd_t(const DevGeom &g, const Real *img, Real *work, Real *out, int *counts,
                        const Real *y_meas, const Real *row_w, hipStream_t stream) {
    constexpr int kSlots = S == 4 ? 4 : 2;
    const Real *copies = nullptr;
    if constexpr (MODE == FwdMode::kPlain || MODE == FwdMode::kSirtResidual) {
        const int nrows = std::max(g.nx, g.ny);
        const int width = padded_width(g.nx, g.ny);
        const size_t total = (size_t)NB * nrows * width;
        const unsigned rows_blocks = (unsigned)std::min<size_t>((total + 255) / 256, 4096);
        const int ti = (nrows + 31) / 32, tp = (width + 31) / 32;
        hipLaunchKernelGGL((pad_kernel<Real, kSlots>), dim3(rows_blocks + (unsigned)(ti * tp * NB)),
                           dim3(32, 8), 0, stream, img, work, g.nx, g.ny, nrows, NB,
                           rows_blocks, ti, tp);
        copies = work;
    }
    dim3 grid((g.nd + kFwdThreads - 1) / kFwdThreads, g.nv);
    hipLaunchKernelGGL((forward_kernel<Real, NB, MODE, S>), grid, dim3(kFwdThreads), 0, stream, g,
                       copies, out, counts, y_meas, row_w);
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

size_t forward_quarter_work_bytes(const DevGeom &g, int nb) {
    const size_t nrows = (size_t)std::max(g.nx, g.ny);
    return (size_t)nb * sizeof(float) * nrows * 4 * (size_t)padded_width(g.nx, g.ny);
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
