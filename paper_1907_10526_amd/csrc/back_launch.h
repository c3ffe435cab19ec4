// Back projection launchers for one beam shape: the batch-chunk, LDS
// capacity and mode dispatch down to one back_kernel instantiation.  Each
// beam and precision has a translation unit (back_<beam>_<f32/f64>.hip) that
// includes this and instantiates launch_back_beam for its beam, so the
// kernels of the three shapes compile in parallel.
#pragma once

#include "kernels.h"

namespace fanproj {
namespace {

template <typename Real, int NB, int CAP>
constexpr bool back_fits() {
    return 2 * (size_t)back_lds_values(NB) * CAP * sizeof(Real) <= kBackLdsLimit;
}

template <typename Real, int NB, int CAP, BackMode MODE, int BEAM>
hipError_t launch_back_t(const DevGeom &g, const Real *sino, Real *img, Real *partial,
                         const Real *col_w, Real relaxation, hipStream_t stream) {
    if constexpr (!back_fits<Real, NB, CAP>()) {
        return hipErrorInvalidValue;  // excluded by back_max_batch
    } else {
        const int groups = partial ? g.back_groups : 1;
        dim3 grid((unsigned)(g.tiles_x * g.tiles_y * groups));
        hipLaunchKernelGGL((back_kernel<Real, NB, CAP, MODE, BEAM>), grid, dim3(kBackThreads), 0,
                           stream, g, sino, img, partial, col_w, relaxation, 0);
        if (groups > 1) {
            const size_t npix = (size_t)g.nx * g.ny;
            const unsigned blocks = (unsigned)std::min<size_t>((npix + 255) / 256, 4096);
            hipLaunchKernelGGL((back_finalize_kernel<Real, NB, MODE>), dim3(blocks), dim3(256), 0,
                               stream, partial, groups, npix, img, col_w, relaxation);
        }
        return hipGetLastError();
    }
}

template <typename Real, int NB, BackMode MODE, int BEAM>
hipError_t launch_back_cap(const DevGeom &g, const Real *sino, Real *img, Real *partial,
                           const Real *col_w, Real relaxation, hipStream_t stream) {
    switch (g.back_cap) {
        case 64: return launch_back_t<Real, NB, 64, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 128: return launch_back_t<Real, NB, 128, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 256: return launch_back_t<Real, NB, 256, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 512: return launch_back_t<Real, NB, 512, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 1024: return launch_back_t<Real, NB, 1024, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename Real, BackMode MODE, int BEAM>
hipError_t launch_back_nb(const DevGeom &g, int nb, const Real *sino, Real *img, Real *partial,
                          const Real *col_w, Real relaxation, hipStream_t stream) {
    switch (nb) {
        case 1: return launch_back_cap<Real, 1, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 2: return launch_back_cap<Real, 2, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 4: return launch_back_cap<Real, 4, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 8: return launch_back_cap<Real, 8, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        default: return hipErrorInvalidValue;
    }
}

// Quarter-turn form (FP32): the back kernel over g (the first quarter of the
// views) with the four view quarters of each of nbi images as 4 nbi images,
// its sums into `partial`, then the rotation-combining finalize.
template <int NBI, int CAP, BackMode MODE, int BEAM>
hipError_t launch_back_quarter_t(const DevGeom &g, const float *sino, float *img, float *partial,
                                 const float *col_w, float relaxation, hipStream_t stream) {
    constexpr int NB = 4 * NBI;
    if constexpr (!back_fits<float, NB, CAP>()) {
        return hipErrorInvalidValue;  // excluded by back_max_batch
    } else {
        const int groups = g.back_groups;
        dim3 grid((unsigned)(g.tiles_x * g.tiles_y * groups));
        hipLaunchKernelGGL((back_kernel<float, NB, CAP, BackMode::kPlain, BEAM>), grid,
                           dim3(kBackThreads), 0, stream, g, sino, img, partial, col_w,
                           relaxation, 1);
        const int n = g.nx;
        dim3 fgrid((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32), (unsigned)NBI);
        hipLaunchKernelGGL((back_finalize_quarter_kernel<MODE>), fgrid, dim3(32, 32), 0, stream,
                           partial, groups, NB, n, img, col_w, relaxation);
        return hipGetLastError();
    }
}

template <int NBI, BackMode MODE, int BEAM>
hipError_t launch_back_quarter_cap(const DevGeom &g, const float *sino, float *img,
                                   float *partial, const float *col_w, float relaxation,
                                   hipStream_t stream) {
    switch (g.back_cap) {
        case 64: return launch_back_quarter_t<NBI, 64, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 128: return launch_back_quarter_t<NBI, 128, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 256: return launch_back_quarter_t<NBI, 256, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 512: return launch_back_quarter_t<NBI, 512, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 1024: return launch_back_quarter_t<NBI, 1024, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        default: return hipErrorInvalidValue;
    }
}

template <BackMode MODE, int BEAM>
hipError_t launch_back_quarter_nb(const DevGeom &g, int nbi, const float *sino, float *img,
                                  float *partial, const float *col_w, float relaxation,
                                  hipStream_t stream) {
    switch (nbi) {
        case 1: return launch_back_quarter_cap<1, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 2: return launch_back_quarter_cap<2, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        default: return hipErrorInvalidValue;
    }
}

// Octant form (FP32, one image): the back kernel over g (the base views) with
// the four rotations and the four reflections of each base view as 8
// images, its sums into `partial`, then the finalize that combines them.
template <int CAP, BackMode MODE, int BEAM>
hipError_t launch_back_octant_t(const DevGeom &g, const float *sino, float *img, float *partial,
                                const float *col_w, float relaxation, hipStream_t stream) {
    if constexpr (!back_fits<float, 8, CAP>()) {
        return hipErrorInvalidValue;  // excluded at geometry creation
    } else {
        const int groups = g.back_groups;
        dim3 grid((unsigned)(g.tiles_x * g.tiles_y * groups));
        hipLaunchKernelGGL((back_kernel<float, 8, CAP, BackMode::kPlain, BEAM>), grid,
                           dim3(kBackThreads), 0, stream, g, sino, img, partial, col_w,
                           relaxation, 1);
        const int n = g.nx;
        dim3 fgrid((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32));
        hipLaunchKernelGGL((back_finalize_octant_kernel<MODE>), fgrid, dim3(32, 32), 0, stream,
                           partial, groups, n, img, col_w, relaxation);
        return hipGetLastError();
    }
}

template <BackMode MODE, int BEAM>
hipError_t launch_back_octant_cap(const DevGeom &g, const float *sino, float *img, float *partial,
                                  const float *col_w, float relaxation, hipStream_t stream) {
    switch (g.back_cap) {
        case 64: return launch_back_octant_t<64, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 128: return launch_back_octant_t<128, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 256: return launch_back_octant_t<256, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        case 512: return launch_back_octant_t<512, MODE, BEAM>(g, sino, img, partial, col_w, relaxation, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <int BEAM>
hipError_t launch_back_octant_beam(const DevGeom &g, BackMode mode, const float *sino, float *img,
                                   float *partial, const float *col_w, float relaxation,
                                   hipStream_t stream) {
    switch (mode) {
        case BackMode::kPlain:
            return launch_back_octant_cap<BackMode::kPlain, BEAM>(g, sino, img, partial, col_w,
                                                                  relaxation, stream);
        case BackMode::kSirtUpdate:
            return launch_back_octant_cap<BackMode::kSirtUpdate, BEAM>(g, sino, img, partial,
                                                                       col_w, relaxation, stream);
        default:
            return hipErrorInvalidValue;
    }
}

template <int BEAM>
hipError_t launch_back_quarter_beam(const DevGeom &g, BackMode mode, int nbi, const float *sino,
                                    float *img, float *partial, const float *col_w,
                                    float relaxation, hipStream_t stream) {
    switch (mode) {
        case BackMode::kPlain:
            return launch_back_quarter_nb<BackMode::kPlain, BEAM>(g, nbi, sino, img, partial,
                                                                  col_w, relaxation, stream);
        case BackMode::kSirtUpdate:
            return launch_back_quarter_nb<BackMode::kSirtUpdate, BEAM>(g, nbi, sino, img, partial,
                                                                       col_w, relaxation, stream);
        default:
            return hipErrorInvalidValue;
    }
}

template <typename Real, int BEAM>
hipError_t launch_back_beam(const DevGeom &g, BackMode mode, int nb, const Real *sino, Real *img,
                            Real *partial, const Real *col_w, Real relaxation,
                            hipStream_t stream) {
    switch (mode) {
        case BackMode::kPlain:
            return launch_back_nb<Real, BackMode::kPlain, BEAM>(g, nb, sino, img, partial, col_w,
                                                                relaxation, stream);
        case BackMode::kSirtUpdate:
            return launch_back_nb<Real, BackMode::kSirtUpdate, BEAM>(g, nb, sino, img, partial,
                                                                     col_w, relaxation, stream);
        case BackMode::kOnes:
            return launch_back_cap<Real, 1, BackMode::kOnes, BEAM>(g, sino, img, partial, col_w,
                                                                   relaxation, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace fanproj

#define FANPROJ_INSTANTIATE_BACK(Real, BEAM)                                                      \
    template hipError_t fanproj::launch_back_beam<Real, BEAM>(                                    \
        const fanproj::DevGeom &, fanproj::BackMode, int, const Real *, Real *, Real *,           \
        const Real *, Real, hipStream_t);
#define FANPROJ_INSTANTIATE_BACK_QUARTER(BEAM)                                                    \
    template hipError_t fanproj::launch_back_quarter_beam<BEAM>(                                  \
        const fanproj::DevGeom &, fanproj::BackMode, int, const float *, float *, float *,        \
        const float *, float, hipStream_t);
#define FANPROJ_INSTANTIATE_BACK_OCTANT(BEAM)                                                     \
    template hipError_t fanproj::launch_back_octant_beam<BEAM>(                                   \
        const fanproj::DevGeom &, fanproj::BackMode, const float *, float *, float *,             \
        const float *, float, hipStream_t);
