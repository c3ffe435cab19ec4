// Back projection: work sizes and the dispatch on the beam shape to the
// launchers instantiated in back_flat.hip, back_arc.hip and back_parallel.hip.
#include "fanproj_internal.h"

namespace fanproj {

template <typename Real>
int back_max_batch(const DevGeom &g) {
    if (g.back_cap <= 0) return 0;
    // two LDS buffers of back_lds_values(nb) arrays of back_cap values
    for (int nb = kMaxBatchChunk; nb >= 1; nb /= 2)
        if (2 * (size_t)back_lds_values(nb) * g.back_cap * sizeof(Real) <= kBackLdsLimit) return nb;
    return 0;
}

template <typename Real>
size_t back_work_bytes(const DevGeom &g, int nb) {
    return g.back_groups > 1 ? (size_t)g.back_groups * nb * g.nx * g.ny * sizeof(Real) : 0;
}

template <typename Real>
hipError_t launch_back(const DevGeom &g, BackMode mode, int nb, const Real *sino, Real *img,
                       Real *partial, const Real *col_w, Real relaxation, hipStream_t stream) {
    switch (g.beam) {
        case FP_FAN_FLAT:
            return launch_back_beam<Real, FP_FAN_FLAT>(g, mode, nb, sino, img, partial, col_w,
                                                       relaxation, stream);
        case FP_FAN_ARC:
            return launch_back_beam<Real, FP_FAN_ARC>(g, mode, nb, sino, img, partial, col_w,
                                                      relaxation, stream);
        case FP_PARALLEL:
            return launch_back_beam<Real, FP_PARALLEL>(g, mode, nb, sino, img, partial, col_w,
                                                       relaxation, stream);
    }
    return hipErrorInvalidValue;
}

size_t back_quarter_work_bytes(const DevGeom &g, int nb) {
    return (size_t)g.back_groups * 4 * nb * g.nx * g.ny * sizeof(float);
}

hipError_t launch_back_quarter(const DevGeom &g, BackMode mode, int nb, const float *sino,
                               float *img, float *partial, const float *col_w, float relaxation,
                               hipStream_t stream) {
    switch (g.beam) {
        case FP_FAN_FLAT:
            return launch_back_quarter_beam<FP_FAN_FLAT>(g, mode, nb, sino, img, partial, col_w,
                                                         relaxation, stream);
        case FP_FAN_ARC:
            return launch_back_quarter_beam<FP_FAN_ARC>(g, mode, nb, sino, img, partial, col_w,
                                                        relaxation, stream);
        case FP_PARALLEL:
            return launch_back_quarter_beam<FP_PARALLEL>(g, mode, nb, sino, img, partial, col_w,
                                                         relaxation, stream);
    }
    return hipErrorInvalidValue;
}

size_t back_octant_work_bytes(const DevGeom &g) {
    return (size_t)g.back_groups * 8 * g.nx * g.ny * sizeof(float);
}

hipError_t launch_back_octant(const DevGeom &g, BackMode mode, const float *sino, float *img,
                              float *partial, const float *col_w, float relaxation,
                              hipStream_t stream) {
    switch (g.beam) {
        case FP_FAN_FLAT:
            return launch_back_octant_beam<FP_FAN_FLAT>(g, mode, sino, img, partial, col_w,
                                                        relaxation, stream);
        case FP_FAN_ARC:
            return launch_back_octant_beam<FP_FAN_ARC>(g, mode, sino, img, partial, col_w,
                                                       relaxation, stream);
        case FP_PARALLEL:
            return launch_back_octant_beam<FP_PARALLEL>(g, mode, sino, img, partial, col_w,
                                                        relaxation, stream);
    }
    return hipErrorInvalidValue;
}

#define FANPROJ_INSTANTIATE(Real)                                                                  \
    template int back_max_batch<Real>(const DevGeom &);                                            \
    template size_t back_work_bytes<Real>(const DevGeom &, int);                                   \
    template hipError_t launch_back<Real>(const DevGeom &, BackMode, int, const Real *, Real *,    \
                                          Real *, const Real *, Real, hipStream_t);
FANPROJ_INSTANTIATE(float)
FANPROJ_INSTANTIATE(double)
#undef FANPROJ_INSTANTIATE

}  // namespace fanproj
