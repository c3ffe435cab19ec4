// CNSF forward and back projection kernels for gfx950 (MI355X).
//
// Every matrix entry is evaluated on the fly (Sec. V-C: no stored system
// matrix, no look-up table) as the closed form of eq. (18):
//
//     A_{(v,m),k} = delta^2 * M_[a, b, tau'](s'),
//
// where a <= b are the two pixel edges projected on the normal of the ray
// through the centre of cell m (eq. (16)), tau' is the effective blur of
// eq. (17) at the pixel's depth L along that ray, and s' is the signed
// distance from the ray to the pixel centre (eq. (13)).
//
// The 3-direction box spline is evaluated as the moving average of the
// 2-direction one over the blur width (the convolution of eq. (9)):
//
//     M_[a,b,c](x) = ( T(x + c/2) - T(x - c/2) ) / c,
//
// with T the antiderivative of the trapezoid M_[a,b].  T is odd about 1/2 and
// its positive half, times b, is
//     Gb(y) = m - (a/2) u^2,   m = min(y, h+),   u = clamp((m - h-) / a, 0, 1)
// (h+ = (a+b)/2, h- = (b-a)/2): a min, one clamped FMA, a square.  No
// truncated power is differenced, so there is no cancellation for near-zero
// a (axis-aligned rays: the rounding of u is then multiplied by a/2) and
// everything runs in FP32.  FP64 is kept for the per-view fan geometry and
// for the offset of a pixel centre from a ray, the one quantity that is a
// small difference of large coordinates.
//
// Forward projection is ray-driven: one thread per detector cell walks the
// rows (or columns) of the image its ray crosses, evaluating the few pixels
// of each row inside the footprint.  Every output is owned by one thread, so
// there are no atomics and no cross-thread reductions.  The walk reads
// zero-padded copies of the image, row-major for rays closer to the y axis and
// transposed for the others, so the pixels of a row are contiguous for every
// ray and consecutive rays read consecutive addresses.
//
// Back projection is a gather: a work-group owns a 16 x 32 pixel tile, two
// pixels per thread.  For each view it stages the per-ray constants and the
// sinogram values of the cells its tile can touch in LDS, then every thread
// sums its pixels' entries from LDS.  Each pixel is written once.
//
// Both kernels sum in two levels (over blocks of 32 rows / views, and over
// blocks) to keep the rounding of 10^3 - 10^4 FP32 terms well under 1e-6
// relative.  Every kernel is instantiated for Real = float (the production
// path) and Real = double (the same arithmetic in FP64 with FP64 tables, for
// finite-difference and adjoint checks).
#include <algorithm>

#include "fanproj_internal.h"

namespace fanproj {
namespace {

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ __forceinline__ double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }

// Per-ray constants of the trapezoid M_[a,b], a <= b.
template <typename Real>
struct Trap {
    Real hab;    // (a + b) / 2
    Real ia;     // 1 / a  (a clamped away from 0)
    Real nhbia;  // -(b - a) / (2a)
    Real ha;     // a / 2
};

// b times the integral over [0, y] (y >= 0) of the centred, unit-mass
// trapezoid.  In FP32 the clamp folds into the FMA's output modifier.
template <typename Real>
__device__ __forceinline__ Real gb(Real y, const Trap<Real> &p) {
    const Real m = fmin(y, p.hab);
    const Real u = clamp01(fma(m, p.ia, p.nhbia));
    return fma(-p.ha * u, u, m);
}

// (2 b hc) * M_[a, b, 2 hc](sp): the blurred footprint up to per-ray and
// per-entry scale factors.
template <typename Real>
__device__ __forceinline__ Real footprint_num(Real sp, Real hc, const Trap<Real> &p) {
    const Real x = fabs(sp);
    const Real y2 = x - hc;
    const Real g1 = gb(x + hc, p);
    const Real g2 = gb(fabs(y2), p);
    return g1 - copysign(g2, y2);
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o));
    return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = min(x, __shfl_xor(x, o));
    return __builtin_amdgcn_readfirstlane(x);
}

constexpr int kSumBlock = 32;

// ---------------------------------------------------------------------------
// Padded image copies for the forward walk, each with NR = max(nx, ny) rows
// (rows past the image are zero, so a wave whose rays march along different
// axes can walk the union of their row ranges):
//   row copy  [nb][NR][nx + 2 pad]: pixel (i, j) at j * (nx + 2 pad) + pad + i
//   col copy  [nb][NR][ny + 2 pad]: pixel (i, j) at i * (ny + 2 pad) + pad + j
// ---------------------------------------------------------------------------
// Row copy of images [0, nb): work item e of the flattened copy.
template <typename Real>
__device__ __forceinline__ void pad_rows_body(const Real *__restrict__ img, Real *__restrict__ rows,
                                              int nx, int ny, int nrows, int nb, size_t first,
                                              size_t stride) {
    const int w = nx + 2 * kFwdPad;
    const size_t per = (size_t)w * nrows;
    const size_t total = per * nb;
    for (size_t e = first; e < total; e += stride) {
        const size_t b = e / per, r = e % per;
        const int j = (int)(r / w), i = (int)(r % w) - kFwdPad;
        rows[e] = (i >= 0 && i < nx && j < ny) ? img[b * (size_t)nx * ny + (size_t)j * nx + i]
                                               : Real(0);
    }
}

// Tiled transpose through LDS: block (32, 8) handles a 32 x 32 tile of the
// column copy (32 copy rows i from i0, 32 padded positions p from p0).
template <typename Real>
__device__ __forceinline__ void pad_cols_tile(const Real *__restrict__ src, Real *__restrict__ dst,
                                              int nx, int ny, int nrows, int i0, int p0,
                                              Real (&tile)[32][33]) {
    const int w = ny + 2 * kFwdPad;
    // read: rows j = p - pad, columns i (coalesced along i)
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int p = p0 + k, j = p - kFwdPad, i = i0 + (int)threadIdx.x;
        Real val = 0;
        if (p < w && j >= 0 && j < ny && i < nx) val = src[(size_t)j * nx + i];
        tile[k][threadIdx.x] = val;
    }
    __syncthreads();
    // write: column copy row i, positions p (coalesced along p)
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int i = i0 + k, p = p0 + (int)threadIdx.x;
        if (i < nrows && p < w) dst[(size_t)i * w + p] = tile[threadIdx.x][k];
    }
    __syncthreads();
}

template <typename Real>
__global__ __launch_bounds__(256) void pad_rows_kernel(const Real *__restrict__ img,
                                                       Real *__restrict__ rows, int nx, int ny,
                                                       int nrows, int nb) {
    pad_rows_body(img, rows, nx, ny, nrows, nb, (size_t)blockIdx.x * blockDim.x + threadIdx.x,
                  (size_t)gridDim.x * blockDim.x);
}

template <typename Real>
__global__ __launch_bounds__(256) void pad_cols_kernel(const Real *__restrict__ img,
                                                       Real *__restrict__ cols, int nx, int ny,
                                                       int nrows) {
    __shared__ Real tile[32][33];
    const int b = blockIdx.z;
    const int w = ny + 2 * kFwdPad;
    pad_cols_tile(img + (size_t)b * nx * ny, cols + (size_t)b * nrows * w, nx, ny, nrows,
                  blockIdx.x * 32, blockIdx.y * 32, tile);
}

// ---------------------------------------------------------------------------
// Forward projection: thread = ray (view blockIdx.y, cell m).
// ---------------------------------------------------------------------------
template <typename Real>
struct RayWalk {
    double S;          // s' at cross index 0 of the current row (FP64)
    double zm, zc;     // s' steps along the march and cross axes
    double izc;        // 1 / zc
    double hq;         // half-span of the footprint along the cross axis, pixels
    Real zcr;          // zc in the arithmetic type
    Real hcr, dhq, dhr;   // half blur at cross index 0 of the row, and its steps
    Trap<Real> trap;
    int nq;            // pixels along the cross axis
    int nr;            // pixels along the march axis
    const Real *base;  // padded copy, cross index 0 of row 0 (image 0)
    size_t row_stride; // values between rows of the copy
    size_t img_stride; // values between images of the copy
};

template <typename Real, int NB, int T, FwdMode MODE>
__device__ __forceinline__ void walk_rows(RayWalk<Real> &w, int r0, int r1, Real (&acc)[NB],
                                          int &nonzero) {
    constexpr bool kLoad = MODE == FwdMode::kPlain || MODE == FwdMode::kSirtResidual;
    const Real *rowp = w.base + (size_t)r0 * w.row_stride;
    for (int rb = r0; rb <= r1; rb += kSumBlock) {
        const int re = min(rb + kSumBlock - 1, r1);
        Real blk[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) blk[b] = 0;
        for (int r = rb; r <= re; ++r, rowp += w.row_stride) {
            // first cross index that can be inside the footprint of this row;
            // clamping keeps the window inside the padded copy (a clamped
            // window lies in the zero margin)
            int q_lo = (int)floor(fma(-w.S, w.izc, -w.hq)) + 1;
            q_lo = min(max(q_lo, -kFwdPad), w.nq + kFwdPad - T);
            const Real sp0 = (Real)fma((double)q_lo, w.zc, w.S);
            const Real hc0 = fma((Real)q_lo, w.dhq, w.hcr);
            w.S += w.zm;
            w.hcr += w.dhr;
            Real cv[NB][T];
            if constexpr (kLoad) {
                const Real *p = rowp + q_lo;
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int t = 0; t < T; ++t) cv[b][t] = p[b * w.img_stride + t];
            } else {
#pragma unroll
                for (int t = 0; t < T; ++t)
                    cv[0][t] = ((unsigned)(q_lo + t) < (unsigned)w.nq && r < w.nr) ? Real(1) : Real(0);
            }
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const Real sp = fma((Real)t, w.zcr, sp0);
                const Real hc = fma((Real)t, w.dhq, hc0);
                const Real e = footprint_num(sp, hc, w.trap) * fast_rcp(hc);
                if constexpr (MODE == FwdMode::kCount) {
                    nonzero += (e != Real(0) && cv[0][t] != Real(0));
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b) blk[b] = fma(e, cv[b][t], blk[b]);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] += blk[b];
    }
}

// Rows whose window is wider than the unrolled variants: same arithmetic,
// a loop over the window with explicit bounds.
template <typename Real, int NB, FwdMode MODE>
__device__ void walk_rows_wide(RayWalk<Real> &w, int T, int r0, int r1, Real (&acc)[NB],
                               int &nonzero) {
    const Real *rowp = w.base + (size_t)r0 * w.row_stride;
    for (int rb = r0; rb <= r1; rb += kSumBlock) {
        const int re = min(rb + kSumBlock - 1, r1);
        Real blk[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) blk[b] = 0;
        for (int r = rb; r <= re; ++r, rowp += w.row_stride) {
            const int q_lo = (int)floor(fma(-w.S, w.izc, -w.hq)) + 1;
            const Real sp0 = (Real)fma((double)q_lo, w.zc, w.S);
            const Real hc0 = fma((Real)q_lo, w.dhq, w.hcr);
            w.S += w.zm;
            w.hcr += w.dhr;
            for (int t = 0; t < T; ++t) {
                const int q = q_lo + t;
                if ((unsigned)q >= (unsigned)w.nq || r >= w.nr) continue;
                const Real sp = fma((Real)t, w.zcr, sp0);
                const Real hc = fma((Real)t, w.dhq, hc0);
                const Real e = footprint_num(sp, hc, w.trap) * fast_rcp(hc);
                if constexpr (MODE == FwdMode::kCount) {
                    nonzero += (e != Real(0));
                } else if constexpr (MODE == FwdMode::kOnes) {
                    blk[0] += e;
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b) blk[b] = fma(e, rowp[q + b * w.img_stride], blk[b]);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] += blk[b];
    }
}

// One block of kFwdThreads consecutive rays of view v, starting at cell
// m_block * kFwdThreads.
template <typename Real, int NB, FwdMode MODE>
__device__ __forceinline__ void forward_block(const DevGeom &G, int v, int m_block,
                                              const Real *__restrict__ rows,
                                              const Real *__restrict__ cols, Real *__restrict__ out,
                                              int *__restrict__ counts,
                                              const Real *__restrict__ y_meas,
                                              const Real *__restrict__ row_w) {
    const RayTables<Real> &tab = ray_tables<Real>(G);
    const int m_thread = m_block * kFwdThreads + threadIdx.x;
    const bool active = m_thread < G.nd;
    // threads past the last cell walk the last ray (their wave needs them for
    // the wave-wide reductions) and write nothing
    const int m = active ? m_thread : G.nd - 1;
    const size_t ray = (size_t)v * G.nd + m;
    const size_t nrays = (size_t)G.nv * G.nd;

    // ---- per-ray frame in FP64 (Sec. II-A, eq. (13)) ----
    const double2 cs = G.views[v];
    const double c = cs.x, sn = cs.y, D = G.dsd;
    const double s = (m - 0.5 * (G.nd - 1)) * G.tau;
    const double R = sqrt(D * D + s * s);
    const double invR = 1.0 / R;
    // ray direction w = (-D u + s e) / R, u = (c, sn), e = (sn, -c);
    // normal w_perp = w rotated by +90 degrees.
    const double wx = (-D * c + s * sn) * invR;
    const double wy = (-D * sn - s * c) * invR;
    const double wpx = -wy, wpy = wx;
    const double px = G.dsc * c, py = G.dsc * sn;
    const double x0 = -0.5 * (G.nx - 1) * G.pixel, y0 = -0.5 * (G.ny - 1) * G.pixel;
    // s'(i, j) and L(i, j) are affine in the pixel indices.
    const double S00 = wpx * (x0 - px) + wpy * (y0 - py);
    const double L00 = wx * (x0 - px) + wy * (y0 - py);
    // March along the image axis closest to the ray; the other ("cross")
    // axis then advances s' by at least delta / sqrt(2) per pixel.
    const bool by_rows = fabs(wy) >= fabs(wx);
    const int nq = by_rows ? G.nx : G.ny, nr = by_rows ? G.ny : G.nx;

    RayWalk<Real> w;
    w.zc = G.pixel * (by_rows ? wpx : wpy);
    w.zm = G.pixel * (by_rows ? wpy : wpx);
    const double lc = G.pixel * (by_rows ? wx : wy);
    const double lm = G.pixel * (by_rows ? wy : wx);
    w.trap.hab = tab.hab[ray];
    w.trap.ia = tab.ia[ray];
    w.trap.nhbia = tab.nhbia[ray];
    w.trap.ha = tab.ha[ray];
    // half effective blur hc = tau'/2 = ghr * R * L, affine in (q, r)
    const double gR = (double)tab.ghr[ray] * R;
    w.dhq = (Real)(gR * lc);
    w.dhr = (Real)(gR * lm);
    w.zcr = (Real)w.zc;
    w.nq = nq;
    w.nr = nr;
    w.row_stride = (size_t)nq + 2 * kFwdPad;
    w.img_stride = w.row_stride * (size_t)max(G.nx, G.ny);
    w.base = (by_rows ? rows : cols) + kFwdPad;

    // Support |s'| < hab + hc, with hc bounded by its value at the far side
    // of the disk containing the image.
    const double lmax = G.dsc * D * invR + G.half_diag;
    const double hw = (double)w.trap.hab + gR * lmax;
    w.izc = 1.0 / w.zc;
    w.hq = hw * fabs(w.izc);
    const int T = (int)floor(2.0 * w.hq) + 1;   // pixels per row that can be hit
    // Rows whose window meets [0, nq): qf(r) = qf0 + r dq is the crossing.
    const double qf0 = -S00 * w.izc, dq = -w.zm * w.izc;
    const double q_lo_lim = -w.hq - 1.0, q_hi_lim = nq + w.hq;
    int r_lo = 0, r_hi = nr - 1;
    if (fabs(dq) > 1e-12) {
        double ra = (q_lo_lim - qf0) / dq, rb = (q_hi_lim - qf0) / dq;
        if (ra > rb) { const double t = ra; ra = rb; rb = t; }
        ra = fmax(ra, -1.0);
        rb = fmin(rb, (double)nr);
        r_lo = max(r_lo, (int)floor(ra));
        r_hi = min(r_hi, (int)ceil(rb));
    } else if (qf0 <= q_lo_lim || qf0 >= q_hi_lim) {
        r_hi = -1;
    }
    if (r_hi < r_lo) { r_lo = nr; r_hi = -1; }

    // The whole wave walks the union of its rays' rows with one window width:
    // control flow stays uniform, and rows or pixels outside a ray's own range
    // read the zero margin or evaluate to zero.
    const int Tw = wave_max(T);
    int r0 = wave_min(r_lo);
    const int r1 = wave_max(r_hi);
    r0 = max(r0, 0);
    w.S = S00 + r0 * w.zm;
    w.hcr = (Real)(gR * (L00 + r0 * lm));

    Real acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0;
    int nonzero = 0;
    if (r0 <= r1) {
        switch (Tw) {
            case 1:
            case 2: walk_rows<Real, NB, 2, MODE>(w, r0, r1, acc, nonzero); break;
            case 3: walk_rows<Real, NB, 3, MODE>(w, r0, r1, acc, nonzero); break;
            case 4: walk_rows<Real, NB, 4, MODE>(w, r0, r1, acc, nonzero); break;
            case 5: walk_rows<Real, NB, 5, MODE>(w, r0, r1, acc, nonzero); break;
            case 6: walk_rows<Real, NB, 6, MODE>(w, r0, r1, acc, nonzero); break;
            case 7:
            case 8: walk_rows<Real, NB, 8, MODE>(w, r0, r1, acc, nonzero); break;
            default: walk_rows_wide<Real, NB, MODE>(w, Tw, r0, r1, acc, nonzero); break;
        }
    }
    if (!active) return;
    const Real wbr = tab.wb[ray];
    if constexpr (MODE == FwdMode::kCount) {
        counts[ray] = nonzero;
    } else if constexpr (MODE == FwdMode::kOnes) {
        const Real sum = acc[0] * wbr;
        out[ray] = sum != Real(0) ? Real(1) / sum : Real(0);
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const Real y = acc[b] * wbr;
            if constexpr (MODE == FwdMode::kPlain) {
                out[b * nrays + ray] = y;
            } else {  // kSirtResidual
                out[b * nrays + ray] = row_w[ray] * (y_meas[b * nrays + ray] - y);
            }
        }
    }
}

template <typename Real, int NB, FwdMode MODE>
__global__ __launch_bounds__(kFwdThreads) void forward_kernel(
    DevGeom G, const Real *__restrict__ rows, const Real *__restrict__ cols,
    Real *__restrict__ out, int *__restrict__ counts, const Real *__restrict__ y_meas,
    const Real *__restrict__ row_w) {
    forward_block<Real, NB, MODE>(G, blockIdx.y, blockIdx.x, rows, cols, out, counts, y_meas,
                                  row_w);
}

// ---------------------------------------------------------------------------
// Back projection: work-group = kBackTileW x kBackTileH pixel tile and one
// contiguous group of views (blockIdx.z of gridDim.z groups).  With one group
// the kernel finishes the pixels itself; with several it writes per-group
// partial sums that back_finalize_kernel adds in group order.
// ---------------------------------------------------------------------------
template <typename Real, int NB, int CAP>
struct BackStage {
    // per-thread share of one view's staged cells (prefetched into registers)
    static constexpr int kPer = (CAP + kBackThreads - 1) / kBackThreads;
    Real invr[kPer], ghr[kPer], hab[kPer], ia[kPer], nhbia[kPer], ha[kPer], w[kPer][NB];
    int4 tc;   // tile entry of the view: M0, cnt, T, H bits
};

template <typename Real, int NB, int CAP>
struct BackLds {
    Real invr[CAP], ghr[CAP], hab[CAP], ia[CAP], nhbia[CAP], ha[CAP], w[NB][CAP];
};

// Staged cell idx holds cell M0 - kBackPad + idx; the kBackPad cells on either
// side of [M0, M0 + cnt) get zero weight and harmless constants.
template <typename Real, int NB, int CAP, BackMode MODE>
__device__ __forceinline__ void back_prefetch(const DevGeom &G, const RayTables<Real> &tab,
                                              const Real *__restrict__ sino, int v, int tile,
                                              int ntiles, size_t nrays,
                                              BackStage<Real, NB, CAP> &st) {
    st.tc = G.tile_cells[(size_t)v * ntiles + tile];
    const int M0 = st.tc.x, cnt = st.tc.y;
#pragma unroll
    for (int k = 0; k < BackStage<Real, NB, CAP>::kPer; ++k) {
        const int idx = (int)threadIdx.x + k * kBackThreads;
        const int c = idx - kBackPad;
        if (c >= 0 && c < cnt) {
            const size_t r = (size_t)v * G.nd + M0 + c;
            st.invr[k] = tab.inv_r[r];
            st.ghr[k] = tab.ghr[r];
            st.hab[k] = tab.hab[r];
            st.ia[k] = tab.ia[r];
            st.nhbia[k] = tab.nhbia[r];
            st.ha[k] = tab.ha[r];
            const Real wb = tab.wb[r];
#pragma unroll
            for (int b = 0; b < NB; ++b)
                st.w[k][b] = (MODE == BackMode::kOnes ? Real(1) : sino[b * nrays + r]) * wb;
        } else {
            st.invr[k] = 0;
            st.ghr[k] = 1;
            st.hab[k] = 1;
            st.ia[k] = 1;
            st.nhbia[k] = 0;
            st.ha[k] = 0;
#pragma unroll
            for (int b = 0; b < NB; ++b) st.w[k][b] = 0;
        }
    }
}

template <typename Real, int NB, int CAP>
__device__ __forceinline__ void back_store(const BackStage<Real, NB, CAP> &st,
                                           BackLds<Real, NB, CAP> &l) {
    const int n = st.tc.y + 2 * kBackPad;
#pragma unroll
    for (int k = 0; k < BackStage<Real, NB, CAP>::kPer; ++k) {
        const int idx = (int)threadIdx.x + k * kBackThreads;
        if (idx < n) {
            l.invr[idx] = st.invr[k];
            l.ghr[idx] = st.ghr[k];
            l.hab[idx] = st.hab[k];
            l.ia[idx] = st.ia[k];
            l.nhbia[idx] = st.nhbia[k];
            l.ha[idx] = st.ha[k];
#pragma unroll
            for (int b = 0; b < NB; ++b) l.w[b][idx] = st.w[k][b];
        }
    }
}

// Entries of one pixel with cells w0 .. w0 + T - 1 of the staged arrays
// (cell m = M0 - kBackPad + w0 + t).  num0 and ln0 are the numerators of s'
// and of R L at the first cell; each further cell steps them by -dnum, +dln.
template <typename Real, int NB, int CAP, bool UNROLLED>
__device__ __forceinline__ void back_window(const BackLds<Real, NB, CAP> &l, int w0, int T,
                                            Real num0, Real dnum, Real ln0, Real dln,
                                            Real (&part)[NB]) {
    const Real *invr = l.invr + w0;
    const Real *ghr = l.ghr + w0;
    const Real *hab = l.hab + w0;
    const Real *ia = l.ia + w0;
    const Real *nhbia = l.nhbia + w0;
    const Real *ha = l.ha + w0;
    auto entry = [&](int t) {
        const Real sp = fma(-(Real)t, dnum, num0) * invr[t];
        const Real hc = fma((Real)t, dln, ln0) * ghr[t];
        const Trap<Real> p{hab[t], ia[t], nhbia[t], ha[t]};
        const Real e = footprint_num(sp, hc, p) * fast_rcp(hc);
#pragma unroll
        for (int b = 0; b < NB; ++b) part[b] = fma(e, l.w[b][w0 + t], part[b]);
    };
    if constexpr (UNROLLED) {
#pragma unroll
        for (int t = 0; t < kBackMaxUnrolled; ++t) {
            if (t >= T) break;  // T is uniform across the work-group
            entry(t);
        }
    } else {
        for (int t = 0; t < T; ++t) entry(t);
    }
}

// One tile (tx, ty) and view group `group` of `groups`.
template <typename Real, int NB, int CAP, BackMode MODE>
__device__ __forceinline__ void back_block(const DevGeom &G, int tx, int ty, int group, int groups,
                                           const Real *__restrict__ sino, Real *__restrict__ img,
                                           Real *__restrict__ partial,
                                           const Real *__restrict__ col_w, Real relaxation) {
    __shared__ BackLds<Real, NB, CAP> lds[2];
    const RayTables<Real> &tab = ray_tables<Real>(G);

    const int tile = ty * G.tiles_x + tx;
    const int ntiles = G.tiles_x * G.tiles_y;
    const size_t npix = (size_t)G.nx * G.ny;
    const size_t nrays = (size_t)G.nv * G.nd;
    const int v_begin = (int)(((long)G.nv * group) / groups);
    const int v_end = (int)(((long)G.nv * (group + 1)) / groups);
    constexpr int P = kBackPixPerThread;
    constexpr int kRowStep = kBackThreads / kBackTileW;
    const int i = tx * kBackTileW + (int)(threadIdx.x % kBackTileW);
    const int j0 = ty * kBackTileH + (int)(threadIdx.x / kBackTileW);
    bool valid[P];
#pragma unroll
    for (int p = 0; p < P; ++p) valid[p] = i < G.nx && j0 + p * kRowStep < G.ny;
    const double xk = (i - 0.5 * (G.nx - 1)) * G.pixel;
    const double yk0 = (j0 - 0.5 * (G.ny - 1)) * G.pixel;
    const double ystep = kRowStep * G.pixel;
    const double D = G.dsd, tau = G.tau, c0 = 0.5 * (G.nd - 1);
    const Real Dr = (Real)D, taur = (Real)tau;
    const float itau = (float)(1.0 / tau), c0f = (float)c0;

    Real acc[P][NB];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[p][b] = 0;

    // software pipeline: view v is computed from lds[v & 1] while view v + 1
    // is loaded into registers; one barrier per view
    BackStage<Real, NB, CAP> st;
    if (v_begin < v_end) {
        back_prefetch<Real, NB, CAP, MODE>(G, tab, sino, v_begin, tile, ntiles, nrays, st);
        back_store<Real, NB, CAP>(st, lds[v_begin & 1]);
    }
    __syncthreads();

    for (int vb = v_begin; vb < v_end; vb += kSumBlock) {
        const int ve = min(vb + kSumBlock, v_end);
        Real blk[P][NB];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int b = 0; b < NB; ++b) blk[p][b] = 0;
        for (int v = vb; v < ve; ++v) {
            const int4 tc = st.tc;
            const int M0 = tc.x, cnt = tc.y, T = tc.z;
            const float H = __int_as_float(tc.w);
            const BackLds<Real, NB, CAP> &l = lds[v & 1];
            if (v + 1 < v_end)
                back_prefetch<Real, NB, CAP, MODE>(G, tab, sino, v + 1, tile, ntiles, nrays, st);

            if (cnt > 0) {
                const double2 cs = G.views[v];
                double ek = xk * cs.y - yk0 * cs.x;             // e . k
                double h = G.dsc - (xk * cs.x + yk0 * cs.y);    // D_sc - u . k
                const double dek = -ystep * cs.x, dh = -ystep * cs.y;
#pragma unroll
                for (int p = 0; p < P; ++p, ek += dek, h += dh) {
                    // the pixel's window: m_lo = ceil((s_k - H) / tau + c0)
                    // with s_k = D (e.k) / h, shifted (never past a non-zero
                    // cell) so that it stays inside the staged cells
                    const float hf = (float)h, ekf = (float)ek;
                    const float sk = (float)D * ekf * fast_rcp(hf);
                    const int m_lo = (int)ceilf(fmaf(sk - H, itau, c0f));
                    const int w0 = min(max(m_lo - M0 + kBackPad, 0),
                                       cnt + 2 * kBackPad - min(T, cnt + 2 * kBackPad));
                    const int m_first = M0 - kBackPad + w0;
                    // s' = (D (e.k) - s_m h) / R_m and R_m L = D h + s_m (e.k) at
                    // the window's first cell in FP64, then steps of one cell
                    const double s_first = (m_first - c0) * tau;
                    const Real num0 = (Real)(D * ek - s_first * h);
                    const Real hr = (Real)h, ekr = (Real)ek;
                    const Real ln0 = fma((Real)s_first, ekr, Dr * hr);
                    const Real dnum = taur * hr, dln = taur * ekr;
                    Real part[NB];
#pragma unroll
                    for (int b = 0; b < NB; ++b) part[b] = 0;
                    if (T <= kBackMaxUnrolled)
                        back_window<Real, NB, CAP, true>(l, w0, T, num0, dnum, ln0, dln, part);
                    else
                        back_window<Real, NB, CAP, false>(l, w0, min(T, cnt + 2 * kBackPad), num0,
                                                          dnum, ln0, dln, part);
#pragma unroll
                    for (int b = 0; b < NB; ++b) blk[p][b] += part[b];
                }
            }
            if (v + 1 < v_end) back_store<Real, NB, CAP>(st, lds[(v + 1) & 1]);
            __syncthreads();
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[p][b] += blk[p][b];
    }

#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!valid[p]) continue;
        const size_t pix = (size_t)(j0 + p * kRowStep) * G.nx + i;
        if (groups > 1) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                partial[((size_t)group * NB + b) * npix + pix] = acc[p][b];
            continue;
        }
        if constexpr (MODE == BackMode::kOnes) {
            const Real sum = acc[p][0];
            img[pix] = sum != Real(0) ? Real(1) / sum : Real(0);
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const Real z = acc[p][b];
                if constexpr (MODE == BackMode::kPlain) {
                    img[b * npix + pix] = z;
                } else {  // kSirtUpdate
                    img[b * npix + pix] += relaxation * col_w[pix] * z;
                }
            }
        }
    }
}

template <typename Real, int NB, int CAP, BackMode MODE>
__global__ __launch_bounds__(kBackThreads) void back_kernel(DevGeom G, const Real *__restrict__ sino,
                                                            Real *__restrict__ img,
                                                            Real *__restrict__ partial,
                                                            const Real *__restrict__ col_w,
                                                            Real relaxation) {
    back_block<Real, NB, CAP, MODE>(G, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.z, sino, img,
                                    partial, col_w, relaxation);
}

// Sum of the view-group partials in group order, then the back kernel's
// epilogue.
template <typename Real, int NB, BackMode MODE>
__global__ __launch_bounds__(256) void back_finalize_kernel(const Real *__restrict__ partial,
                                                            int groups, size_t npix,
                                                            Real *__restrict__ img,
                                                            const Real *__restrict__ col_w,
                                                            Real relaxation) {
    for (size_t pix = (size_t)blockIdx.x * blockDim.x + threadIdx.x; pix < npix;
         pix += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            Real z = 0;
            for (int g = 0; g < groups; ++g) z += partial[((size_t)g * NB + b) * npix + pix];
            if constexpr (MODE == BackMode::kOnes) {
                img[pix] = z != Real(0) ? Real(1) / z : Real(0);
            } else if constexpr (MODE == BackMode::kPlain) {
                img[b * npix + pix] = z;
            } else {
                img[b * npix + pix] += relaxation * col_w[pix] * z;
            }
        }
    }
}

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
    back_block<float, 1, CAP, BackMode::kSirtUpdate>(J.g, local % J.g.tiles_x, local / J.g.tiles_x,
                                                    0, 1, J.work, J.image_out, nullptr, J.col_w,
                                                    J.relaxation);
}

// ------------------------------- launchers ---------------------------------

template <typename Real, int NB, FwdMode MODE>
hipError_t launch_fwd_t(const DevGeom &g, const Real *img, Real *work, Real *out, int *counts,
                        const Real *y_meas, const Real *row_w, hipStream_t stream) {
    const Real *rows = nullptr, *cols = nullptr;
    if constexpr (MODE == FwdMode::kPlain || MODE == FwdMode::kSirtResidual) {
        const int nrows = std::max(g.nx, g.ny);
        Real *wr = work;
        Real *wc = work + (size_t)NB * nrows * (g.nx + 2 * kFwdPad);
        const size_t total = (size_t)NB * nrows * (g.nx + 2 * kFwdPad);
        const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 65535);
        hipLaunchKernelGGL(pad_rows_kernel<Real>, dim3(blocks), dim3(256), 0, stream, img, wr, g.nx,
                           g.ny, nrows, NB);
        dim3 tgrid((nrows + 31) / 32, (g.ny + 2 * kFwdPad + 31) / 32, NB);
        hipLaunchKernelGGL(pad_cols_kernel<Real>, tgrid, dim3(32, 8), 0, stream, img, wc, g.nx,
                           g.ny, nrows);
        rows = wr;
        cols = wc;
    }
    dim3 grid((g.nd + kFwdThreads - 1) / kFwdThreads, g.nv);
    hipLaunchKernelGGL((forward_kernel<Real, NB, MODE>), grid, dim3(kFwdThreads), 0, stream, g,
                       rows, cols, out, counts, y_meas, row_w);
    return hipGetLastError();
}

template <typename Real, FwdMode MODE>
hipError_t launch_fwd_nb(const DevGeom &g, int nb, const Real *img, Real *work, Real *out,
                         int *counts, const Real *y_meas, const Real *row_w, hipStream_t stream) {
    switch (nb) {
        case 1: return launch_fwd_t<Real, 1, MODE>(g, img, work, out, counts, y_meas, row_w, stream);
        case 2: return launch_fwd_t<Real, 2, MODE>(g, img, work, out, counts, y_meas, row_w, stream);
        case 4: return launch_fwd_t<Real, 4, MODE>(g, img, work, out, counts, y_meas, row_w, stream);
        case 8: return launch_fwd_t<Real, 8, MODE>(g, img, work, out, counts, y_meas, row_w, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename Real, int NB, int CAP>
constexpr bool back_fits() {
    return 2 * (size_t)(kBackRayParams + NB) * CAP * sizeof(Real) <= kBackLdsLimit;
}

template <typename Real, int NB, int CAP, BackMode MODE>
hipError_t launch_back_t(const DevGeom &g, const Real *sino, Real *img, Real *partial,
                         const Real *col_w, Real relaxation, hipStream_t stream) {
    if constexpr (!back_fits<Real, NB, CAP>()) {
        return hipErrorInvalidValue;  // excluded by back_max_batch
    } else {
        const int groups = partial ? g.back_groups : 1;
        dim3 grid(g.tiles_x, g.tiles_y, groups);
        hipLaunchKernelGGL((back_kernel<Real, NB, CAP, MODE>), grid, dim3(kBackThreads), 0, stream,
                           g, sino, img, partial, col_w, relaxation);
        if (groups > 1) {
            const size_t npix = (size_t)g.nx * g.ny;
            const unsigned blocks = (unsigned)std::min<size_t>((npix + 255) / 256, 4096);
            hipLaunchKernelGGL((back_finalize_kernel<Real, NB, MODE>), dim3(blocks), dim3(256), 0,
                               stream, partial, groups, npix, img, col_w, relaxation);
        }
        return hipGetLastError();
    }
}

template <typename Real, int NB, BackMode MODE>
hipError_t launch_back_cap(const DevGeom &g, const Real *sino, Real *img, Real *partial,
                           const Real *col_w, Real relaxation, hipStream_t stream) {
    switch (g.back_cap) {
        case 64: return launch_back_t<Real, NB, 64, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        case 128: return launch_back_t<Real, NB, 128, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        case 256: return launch_back_t<Real, NB, 256, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        case 512: return launch_back_t<Real, NB, 512, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        case 1024: return launch_back_t<Real, NB, 1024, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename Real, BackMode MODE>
hipError_t launch_back_nb(const DevGeom &g, int nb, const Real *sino, Real *img, Real *partial,
                          const Real *col_w, Real relaxation, hipStream_t stream) {
    switch (nb) {
        case 1: return launch_back_cap<Real, 1, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        case 2: return launch_back_cap<Real, 2, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        case 4: return launch_back_cap<Real, 4, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        case 8: return launch_back_cap<Real, 8, MODE>(g, sino, img, partial, col_w, relaxation, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename Real>
size_t forward_work_bytes(const DevGeom &g, int nb) {
    const size_t nrows = (size_t)std::max(g.nx, g.ny);
    return (size_t)nb * sizeof(Real) * nrows * ((size_t)(g.nx + 2 * kFwdPad) + (g.ny + 2 * kFwdPad));
}

template <typename Real>
int back_max_batch(const DevGeom &g) {
    if (g.back_cap <= 0) return 0;
    // two LDS buffers of (kBackRayParams + nb) arrays of back_cap values
    for (int nb = kMaxBatchChunk; nb >= 1; nb /= 2)
        if (2 * (size_t)(kBackRayParams + nb) * g.back_cap * sizeof(Real) <= kBackLdsLimit) return nb;
    return 0;
}

template <typename Real>
size_t back_work_bytes(const DevGeom &g, int nb) {
    return g.back_groups > 1 ? (size_t)g.back_groups * nb * g.nx * g.ny * sizeof(Real) : 0;
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
            return launch_fwd_t<Real, 1, FwdMode::kOnes>(g, img, work, out, counts, y_meas, row_w,
                                                         stream);
        case FwdMode::kCount:
            return launch_fwd_t<Real, 1, FwdMode::kCount>(g, img, work, out, counts, y_meas, row_w,
                                                          stream);
    }
    return hipErrorInvalidValue;
}

template <typename Real>
hipError_t launch_back(const DevGeom &g, BackMode mode, int nb, const Real *sino, Real *img,
                       Real *partial, const Real *col_w, Real relaxation, hipStream_t stream) {
    switch (mode) {
        case BackMode::kPlain:
            return launch_back_nb<Real, BackMode::kPlain>(g, nb, sino, img, partial, col_w,
                                                          relaxation, stream);
        case BackMode::kSirtUpdate:
            return launch_back_nb<Real, BackMode::kSirtUpdate>(g, nb, sino, img, partial, col_w,
                                                               relaxation, stream);
        case BackMode::kOnes:
            return launch_back_cap<Real, 1, BackMode::kOnes>(g, sino, img, partial, col_w,
                                                             relaxation, stream);
    }
    return hipErrorInvalidValue;
}

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

#define FANPROJ_INSTANTIATE(Real)                                                                  \
    template size_t forward_work_bytes<Real>(const DevGeom &, int);                                \
    template int back_max_batch<Real>(const DevGeom &);                                            \
    template size_t back_work_bytes<Real>(const DevGeom &, int);                                   \
    template hipError_t launch_forward<Real>(const DevGeom &, FwdMode, int, const Real *, Real *,  \
                                             Real *, int *, const Real *, const Real *,            \
                                             hipStream_t);                                          \
    template hipError_t launch_back<Real>(const DevGeom &, BackMode, int, const Real *, Real *,    \
                                          Real *, const Real *, Real, hipStream_t);
FANPROJ_INSTANTIATE(float)
FANPROJ_INSTANTIATE(double)
#undef FANPROJ_INSTANTIATE

}  // namespace fanproj
