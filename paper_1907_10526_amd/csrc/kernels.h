// CNSF forward and back projection kernels for gfx950 (MI355X): the device
// code shared by the translation units that instantiate and launch it.
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
// (h+ = (a+b)/2, h- = (b-a)/2); footprint_num takes the two terms of the
// moving average together (a median, a clamped FMA and a square each).  No
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
// Both kernels sum in two levels (over blocks of 64 rows / 32 views, and over
// blocks) to keep the rounding of 10^3 - 10^4 FP32 terms well under 1e-6
// relative.  Every kernel is instantiated for Real = float (the production
// path) and Real = double (the same arithmetic in FP64 with FP64 tables, for
// finite-difference and adjoint checks).
#pragma once

#include <algorithm>
#include <type_traits>

#include "fanproj_internal.h"

namespace fanproj {
namespace {

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ __forceinline__ double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }
// min(x, c) for finite x, c: the median of x, c and the most negative finite
// float, which (unlike fmin) takes an operand loaded from memory as it is
__device__ __forceinline__ float fmin_finite(float x, float c) {
    return __builtin_amdgcn_fmed3f(x, c, -3.40282347e38f);
}
__device__ __forceinline__ double fmin_finite(double x, double c) { return fmin(x, c); }

// Per-ray constants of the trapezoid M_[a,b], a <= b.
template <typename Real>
struct Trap {
    Real hab;    // (a + b) / 2
    Real ia;     // 1 / a  (a clamped away from 0)
    Real nhbia;  // -(b - a) / (2a)
    Real ha;     // a / 2
};

// clamp(y, -h, h) for finite y, h >= 0
__device__ __forceinline__ float clamp_sym(float y, float h) {
    return __builtin_amdgcn_fmed3f(y, -h, h);
}
__device__ __forceinline__ double clamp_sym(double y, double h) { return fmin(fmax(y, -h), h); }

// (2 b hc) * M_[a, b, 2 hc](sp): the blurred footprint up to per-ray and
// per-entry scale factors.  With G the odd function whose value at y >= 0 is
// b times the integral over [0, y] of the centred, unit-mass trapezoid,
//   G(y) = m - (a/2) u^2,  m = clamp(y, -hab, hab),  u = clamp((|m| - h-) / a, 0, 1)
// for y >= 0 and odd, the footprint is G(x + hc) - G(x - hc), x = |s'|; with
// both terms together it is (m1 - m2) - (a/2) (u1^2 - sign(x - hc) u2^2).
// In FP32 the clamps fold into medians and the FMA's output modifier.
template <typename Real>
__device__ __forceinline__ Real footprint_num(Real sp, Real hc, const Trap<Real> &p) {
    const Real x = fabs(sp);
    const Real y2 = x - hc;
    const Real m1 = fmin_finite(x + hc, p.hab);   // x + hc >= 0
    const Real m2 = clamp_sym(y2, p.hab);
    const Real u1 = clamp01(fma(m1, p.ia, p.nhbia));
    const Real u2 = clamp01(fma(fabs(m2), p.ia, p.nhbia));
    const Real dq = fma(copysign(u2, y2), -u2, u1 * u1);
    return fma(-p.ha, dq, m1 - m2);
}

// Waves per SIMD the projection kernels are compiled for: eight (at most 64
// VGPRs) for one FP32 image, the occupancy their launches are sized for, and
// for four (the back projection's quarter-turn form, whose 8 waves per SIMD
// then run in one round: measured 8 % faster than at its natural 5 waves
// despite a few spilled registers); no bound for the other batched and the
// FP64 variants, which need more registers.
constexpr int min_waves(int nb, size_t real_bytes) {
    return (nb == 1 || nb == 4) && real_bytes == 4 ? 8 : 1;
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

constexpr int kSumBlock = 32;        // views per partial sum of the back projection
constexpr int kFwdBlockRows = 64;    // rows per block of the forward walk

// ---------------------------------------------------------------------------
// Padded image copies for the forward walk, row-major and transposed, each
// with NR = max(nx, ny) rows of W = NR + 2 pad values (rows and values past
// the image are zero, so a wave whose rays march along different axes can
// walk the union of their row ranges with one clamp bound), interleaved row
// by row: copies [nb][NR][2][W], so that row r of either copy is at one
// address common to the wave plus a small per-lane offset (0 or W):
//   row copy  (slot 0): pixel (i, j) at (j * 2 + 0) * W + pad + i
//   col copy  (slot 1): pixel (i, j) at (i * 2 + 1) * W + pad + j
// ---------------------------------------------------------------------------
// Row copy (slot 0) of images [0, nb): work item e of the flattened copy.
template <typename Real>
__device__ __forceinline__ void pad_rows_body(const Real *__restrict__ img,
                                              Real *__restrict__ copies, int nx, int ny,
                                              int nrows, int nb, size_t first, size_t stride) {
    const int w = padded_width(nx, ny);
    const size_t total = (size_t)w * nrows * nb;
    for (size_t e = first; e < total; e += stride) {
        const size_t row = e / w;    // b * nrows + j
        const int j = (int)(row % nrows), i = (int)(e % w) - kFwdPad;
        const size_t b = row / nrows;
        copies[row * 2 * w + e % w] =
            (i >= 0 && i < nx && j < ny) ? img[b * (size_t)nx * ny + (size_t)j * nx + i] : Real(0);
    }
}

// Tiled transpose through LDS: block (32, 8) handles a 32 x 32 tile of the
// column copy (32 copy rows i from i0, 32 padded positions p from p0); dst is
// the image's column copy (slot 1 of its first row), rows 2 W apart.
template <typename Real>
__device__ __forceinline__ void pad_cols_tile(const Real *__restrict__ src, Real *__restrict__ dst,
                                              int nx, int ny, int nrows, int i0, int p0,
                                              Real (&tile)[32][33]) {
    const int w = padded_width(nx, ny);
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
        if (i < nrows && p < w) dst[(size_t)i * 2 * w + p] = tile[threadIdx.x][k];
    }
    __syncthreads();
}

// Both padded copies of a batch in one launch of 32 x 8 blocks: the first
// rows_blocks blocks stride over the row copies, each further block
// transposes one 32 x 32 tile of one image's column copy (ti x tp tiles per
// image).
template <typename Real>
__global__ __launch_bounds__(256) void pad_kernel(const Real *__restrict__ img,
                                                  Real *__restrict__ copies, int nx, int ny,
                                                  int nrows, int nb, unsigned rows_blocks, int ti,
                                                  int tp) {
    __shared__ Real tile[32][33];
    const int tid = threadIdx.y * 32 + threadIdx.x;
    if (blockIdx.x < rows_blocks) {
        pad_rows_body(img, copies, nx, ny, nrows, nb, (size_t)blockIdx.x * 256 + tid,
                      (size_t)rows_blocks * 256);
        return;
    }
    const int t = (int)(blockIdx.x - rows_blocks);
    const int b = t / (ti * tp), k = t % (ti * tp);
    const int w = padded_width(nx, ny);
    pad_cols_tile(img + (size_t)b * nx * ny, copies + ((size_t)b * nrows * 2 + 1) * w, nx, ny,
                  nrows, (k % ti) * 32, (k / ti) * 32, tile);
}

// ---------------------------------------------------------------------------
// Forward projection: thread = ray (view blockIdx.x, cell m).
// ---------------------------------------------------------------------------
template <typename Real>
struct RayWalk {
    // X = 1 - s'(cross index 0) / zc - hq on a row, in FP64: a window of
    // half span hq starts at cross index floor(X), and s' there equals
    // zc (1 - hq - frac(X)).  X1 is 1 - s'(cross index 0) / zc on row r0.
    double X1, dX;     // and its step per row
    float hq;          // half span of the ray's support along the cross axis
    Real zcr;          // zc in the arithmetic type
    Real dhq, dhr;     // steps of the half blur along the cross axis and per row
    Real hc0, dhc;     // half blur at cross index 0 of row r0, and its step per row
    // Half span a window on row r needs: (hab + hc_fix + g L) / |zc| with L
    // the depth of the window's pixels, at most the ray's depth where it
    // crosses the row plus the window's half extent: hq_row(r) = hqa + hqb
    // (r - r0), affine in r, capped at hq.  A bound, so FP32 with a relative
    // margin.
    float hqa, hqb;
    Trap<Real> trap;
    int nq;            // pixels along the cross axis
    int width;         // length of a padded copy's rows (uniform)
    // Offsets (values) within a row pair of the copies this ray reads: one
    // read for S = 1 (its own axis' copy, 0 or width); for S = 4, the four
    // quarter-turn rotations (forward_block): q = 0 its own copy on row r,
    // q = 1 the other copy on row r read mirrored, q = 2 the other copy on
    // row nr-1-r, q = 3 its own copy on row nr-1-r read mirrored.
    int qoff[4];
    int nr;            // pixels along the march axis
    int r0;            // first row of the walk
    const Real *base;  // the interleaved copies (image 0, row 0), uniform
    size_t row_stride; // values between row pairs (2 width)
    size_t img_stride; // values between images
};

// Row stepper of walk_block.  FP64 (the FP64 instantiation): X itself.
// FP32: X + kFwdPad in 32.32 fixed point, re-anchored from the FP64 X at the
// start of every block of kFwdBlockRows rows (so its drift stays below
// kFwdBlockRows * 2^-33 pixel); one 64-bit integer add per row, the high word is
// the padded cross index of the window start and the low word its fraction.
template <typename Real>
struct RowStepper {
    double X;
    __device__ void start(double X0) { X = X0; }
    // padded window start p (clamped to [0, p_max]) and fraction of X
    __device__ __forceinline__ void row(unsigned p_max, unsigned &p, Real &frac) {
        const double fl = floor(X);
        const int q = (int)fl;
        p = (unsigned)min(max(q, -kFwdPad), (int)p_max - kFwdPad) + kFwdPad;
        frac = (Real)(X - fl);
    }
    __device__ __forceinline__ void next(double dX) { X += dX; }
};
template <>
struct RowStepper<float> {
    double X;                // FP64 X at the start of the block
    unsigned long long q;    // X + kFwdPad in 32.32 fixed point (two's complement)
    unsigned long long dq;   // its step per row
    __device__ void start(double X0) { X = X0; }
    __device__ void anchor(double dX) {
        const double xb = X + kFwdPad, fl = floor(xb);
        q = (unsigned long long)((long long)fl * 4294967296LL) +
            (unsigned)((xb - fl) * 4294967296.0);
        dq = (unsigned long long)(long long)rint(dX * 4294967296.0);   // |dX| <= 1
    }
    // (a negative X + kFwdPad wraps to a large unsigned value and clamps to
    // p_max, a window in the zero margin on the far side)
    __device__ __forceinline__ void row(unsigned p_max, unsigned &p, float &frac) {
        p = min((unsigned)(q >> 32), p_max);
        frac = (float)(unsigned)q;   // the fraction in units of 2^-32
    }
    // One 64-bit add (written out: the compiler's loop strength reduction
    // otherwise splits the stepper into several induction variables).
    __device__ __forceinline__ void next(double) {
        asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(q) : "v"(q), "v"(dq));
    }
};

// Rows rb .. re with windows of T pixels.  Xb is X on row rb for the
// block's half span, whose s' at frac(X) = 0 is sp_top; hcp is the half blur
// at padded cross index 0 of row rb.  Sums into blk: NB images, and for
// S = 4 the four rotations of each (accumulator q NB + b).
template <typename Real, int NB, int T, FwdMode MODE, int S>
__device__ __forceinline__ void walk_block(const RayWalk<Real> &w, double Xb, Real sp_top,
                                           Real hcp, int rb, int re, Real (&blk)[NB * S],
                                           int &nonzero) {
    constexpr int K = NB * S;
    constexpr bool kLoad = MODE == FwdMode::kPlain || MODE == FwdMode::kSirtResidual;
    constexpr bool kFixed = std::is_same<Real, float>::value;
    static_assert(S == 1 || kLoad, "rotations are read only by the image modes");
    // the window start, clamped so that the window stays inside the padded
    // copy (a clamped window, and the unclamped one it replaces, lie in the
    // zero margin: its s' is then immaterial)
    const unsigned p_max = (unsigned)(w.width - T);
    // s' at the window start is zc (1 - hq - frac(X)); in fixed point frac
    // arrives in units of 2^-32
    const Real zfrac = kFixed ? -w.zcr * Real(2.3283064365386963e-10) : -w.zcr;
    // row r of every copy starts at one address common to the wave; the
    // lane's window is a small byte offset from it (S = 4: and row nr-1-r,
    // walked backwards)
    const size_t stride = w.row_stride;
    const Real *rowp = w.base + (size_t)rb * stride;
    // (S = 4: the image is square, so nr is the same for every lane: saying
    // so keeps the mirrored row's pointer in scalar registers)
    const int nr_u = S == 4 ? __builtin_amdgcn_readfirstlane(w.nr) : w.nr;
    const Real *mrowp = S == 4 ? w.base + (size_t)(nr_u - 1 - rb) * stride : rowp;

    // the window's pixel values of row r (rows rp and mp) starting at p
    auto load = [&](Real (&cv)[K][T], const Real *rp, const Real *mp, unsigned p, int r) {
        if constexpr (kLoad) {
#pragma unroll
            for (int q = 0; q < S; ++q) {
                // reads q = 1, 3 run backwards from the mirrored position
                // W - 1 - p (negative immediate offsets)
                const bool mir = q & 1;
                const Real *pp = reinterpret_cast<const Real *>(
                    reinterpret_cast<const char *>(q < 2 ? rp : mp) +
                    (unsigned)(w.qoff[q] + (mir ? w.width - 1 - (int)p : (int)p)) *
                        (unsigned)sizeof(Real));
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int t = 0; t < T; ++t)
                        cv[q * NB + b][t] = pp[b * w.img_stride + (mir ? -t : t)];
            }
        } else {
#pragma unroll
            for (int t = 0; t < T; ++t)
                cv[0][t] = ((unsigned)((int)p - kFwdPad + t) < (unsigned)w.nq && r < w.nr)
                               ? Real(1) : Real(0);
        }
    };
    // the entries of one row (window at p, fraction frac, half blur hcr at
    // padded cross index 0)
    auto entries = [&](const Real (&cv)[K][T], unsigned p, Real frac, Real hcr) {
        const Real sp0 = fma(zfrac, frac, sp_top);
        const Real hc0 = fma((Real)p, w.dhq, hcr);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            // (t == 0 spelled out: an FMA by zero does not fold)
            const Real sp = t == 0 ? sp0 : fma((Real)t, w.zcr, sp0);
            const Real hc = t == 0 ? hc0 : fma((Real)t, w.dhq, hc0);
            if constexpr (MODE == FwdMode::kCount) {
                // the entry is non-zero on the support |s'| < hab + hc
                nonzero += (fabs(sp) < w.trap.hab + hc && cv[0][t] != Real(0));
            } else {
                const Real e = footprint_num(sp, hc, w.trap) * fast_rcp(hc);
#pragma unroll
                for (int k = 0; k < K; ++k) blk[k] = fma(e, cv[k][t], blk[k]);
            }
        }
    };

    RowStepper<Real> X;
    X.start(Xb);
    if constexpr (kFixed) X.anchor(w.dX);
    for (int r = rb; r <= re; ++r) {
        unsigned p;
        Real frac;
        X.row(p_max, p, frac);
        Real cv[K][T];
        load(cv, rowp, mrowp, p, r);
        entries(cv, p, frac, hcp);
        hcp += w.dhr;
        X.next(w.dX);
        rowp += stride;
        if constexpr (S == 4) mrowp -= stride;
    }
}

// Windows wider than the unrolled variants: same arithmetic, a loop over the
// window with explicit bounds, X in FP64.
template <typename Real, int NB, FwdMode MODE, int S>
__device__ void walk_block_wide(const RayWalk<Real> &w, int T, double X, Real sp_top, Real hcp,
                                int rb, int re, Real (&blk)[NB * S], int &nonzero) {
    const Real *rowp = w.base + (size_t)rb * w.row_stride;
    const Real *mrowp = S == 4 ? w.base + (size_t)(w.nr - 1 - rb) * w.row_stride : rowp;
    for (int r = rb; r <= re;
         ++r, rowp += w.row_stride, mrowp -= S == 4 ? w.row_stride : 0, X += w.dX, hcp += w.dhr) {
        const double fl = floor(X);
        const int q_lo = (int)fl;
        const Real sp0 = fma(-w.zcr, (Real)(X - fl), sp_top);
        const Real hc0 = fma((Real)(q_lo + kFwdPad), w.dhq, hcp);
        for (int t = 0; t < T; ++t) {
            const int q = q_lo + t;
            if ((unsigned)q >= (unsigned)w.nq || r >= w.nr) continue;
            const Real sp = fma((Real)t, w.zcr, sp0);
            const Real hc = fma((Real)t, w.dhq, hc0);
            if constexpr (MODE == FwdMode::kCount) {
                nonzero += (fabs(sp) < w.trap.hab + hc);
                continue;
            }
            const Real e = footprint_num(sp, hc, w.trap) * fast_rcp(hc);
            if constexpr (MODE == FwdMode::kOnes) {
                blk[0] += e;
            } else {
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    // (reads k = 1, 3 mirrored, as in walk_block)
                    const int x = kFwdPad + q;
                    const Real *pk =
                        (k < 2 ? rowp : mrowp) + w.qoff[k] + ((k & 1) ? w.width - 1 - x : x);
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        blk[k * NB + b] = fma(e, pk[b * w.img_stride], blk[k * NB + b]);
                }
            }
        }
    }
}

// The walk over rows r0 .. r1 in blocks of kFwdBlockRows rows.  Each block's
// window width is the wave's largest need over the block: the blur grows
// with depth along the ray, so blocks on the source side take narrower
// windows than the ray's deepest row would.
template <typename Real, int NB, FwdMode MODE, int S, int TMAX>
__device__ __forceinline__ void walk_rows(const RayWalk<Real> &w, int r_first, int r1,
                                          Real (&acc)[NB * S], int &nonzero) {
    constexpr int K = NB * S;
    for (int rb = r_first; rb <= r1; rb += kFwdBlockRows) {
        const int re = min(rb + kFwdBlockRows - 1, r1);
        // the block's half span (a lane whose ray misses the block's rows
        // reads only the zero margin, whatever its window)
        const float ha = fmaf((float)(rb - w.r0), w.hqb, w.hqa);
        const float hb = fmaf((float)(re - w.r0), w.hqb, w.hqa);
        const float hqk = fmaxf(0.0f, fminf(w.hq, fmaxf(ha, hb)));
        const int Tb = max(wave_max((int)floorf(2.0f * hqk) + 1), 1);
        const double Xb = fma((double)(rb - w.r0), w.dX, w.X1) - (double)hqk;
        // (the same hqk in both: X and s' at the window start stay consistent)
        const Real sp_top = w.zcr * (Real)(1.0 - (double)hqk);
        // half blur at padded cross index 0 of row rb
        const Real hcp = fma(-(Real)kFwdPad, w.dhq, fma((Real)(rb - w.r0), w.dhc, w.hc0));
        Real blk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) blk[k] = 0;
        switch (Tb) {
            case 1:
            case 2: walk_block<Real, NB, 2, MODE, S>(w, Xb, sp_top, hcp, rb, re, blk, nonzero); break;
            case 3: walk_block<Real, NB, 3, MODE, S>(w, Xb, sp_top, hcp, rb, re, blk, nonzero); break;
            case 4: walk_block<Real, NB, 4, MODE, S>(w, Xb, sp_top, hcp, rb, re, blk, nonzero); break;
            // (windows wider than TMAX take the loop: the quarter-turn form
            // holds four loads per pixel, and a narrower widest window keeps
            // its registers for more waves)
            case 5:
                if constexpr (TMAX >= 5) {
                    walk_block<Real, NB, 5, MODE, S>(w, Xb, sp_top, hcp, rb, re, blk, nonzero);
                    break;
                }
                [[fallthrough]];
            case 6:
                if constexpr (TMAX >= 6) {
                    walk_block<Real, NB, 6, MODE, S>(w, Xb, sp_top, hcp, rb, re, blk, nonzero);
                    break;
                }
                [[fallthrough]];
            case 7:
            case 8:
                if constexpr (TMAX >= 8) {
                    walk_block<Real, NB, 8, MODE, S>(w, Xb, sp_top, hcp, rb, re, blk, nonzero);
                    break;
                }
                [[fallthrough]];
            default:
                walk_block_wide<Real, NB, MODE, S>(w, Tb, Xb, sp_top, hcp, rb, re, blk, nonzero);
                break;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += blk[k];
    }
}

// One work-group of fwd_rays_per_block(S) consecutive rays of view v,
// starting at cell m_block times that.
//
// S = 4 (square image, views in quarter-turn quadruples v + k nv, k < 4,
// where G holds the nv views of the first quarter): the entries of view
// v + k nv on the image c equal those of view v on c rotated by k quarter
// turns, (c o R^k)(i, j) with R(i, j) = (n-1-j, i), so one walk evaluates
// every entry once for the four views.  Walking row r of its own axis' copy
// at cross position x, a ray finds the four rotations at
//   k = 0: its own copy, row r, x
//   rows:    k = 1 column copy, row n-1-r, x;  2 row copy, row n-1-r, mirrored x;
//            k = 3 column copy, row r, mirrored x
//   columns: k = 1 row copy, row r, mirrored x;  2 column copy, row n-1-r,
//            mirrored x;  k = 3 row copy, row n-1-r, x
// (mirrored x = W - 1 - x, a read running backwards), so the reads q = 0, 1
// share row r and q = 2, 3 row n-1-r (RayWalk::qoff).  The outputs are
// [nb][4][nv][nd]: image b's sinogram of 4 nv views.
// TMAX: the widest window walked with an unrolled row (wider ones take the
// loop of walk_block_wide): 8 for the plain walk, 6 or 4 for the quarter-turn
// walk (4 when no window of the geometry is wider, DevGeom::fwd_window).
template <typename Real, int NB, FwdMode MODE, int S, int TMAX = (S == 1 ? 8 : 6)>
__device__ __forceinline__ void forward_block(const DevGeom &G, int v, int m_block,
                                              const Real *__restrict__ copies,
                                              Real *__restrict__ out,
                                              int *__restrict__ counts,
                                              const Real *__restrict__ y_meas,
                                              const Real *__restrict__ row_w) {
    const RayTables<Real> &tab = ray_tables<Real>(G);
    // S = 4: the work-group's kParts parts walk consecutive shares of the row
    // blocks of the same rays (waves w and w + kRays / 64 hold the same rays,
    // so their row ranges agree)
    constexpr int kParts = S == 4 ? kFwdQuarterParts : 1;
    constexpr int kRays = kFwdThreads / kParts;
    // (kRays is a multiple of the wave size, so the part is uniform across
    // the wave; saying so keeps the row loop's pointers and bounds in scalar
    // registers)
    const int part = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kRays);
    const int m_thread = m_block * kRays + (int)threadIdx.x % kRays;
    const bool active = m_thread < G.nd;
    // threads past the last cell walk the last ray (their wave needs them for
    // the wave-wide reductions) and write nothing
    const int m = active ? m_thread : G.nd - 1;
    const size_t ray = (size_t)v * G.nd + m;
    const size_t nrays = (size_t)G.nv * G.nd;

    // ---- per-ray frame in FP64 (Sec. II-A, eq. (13)) ----
    const double2 cs = G.views[v];
    const double c = cs.x, sn = cs.y, D = G.dsd;
    const double s = (m - 0.5 * (G.nd - 1)) * G.pitch;
    const double x0 = -0.5 * (G.nx - 1) * G.pixel, y0 = -0.5 * (G.ny - 1) * G.pixel;
    // ray direction w (source towards detector) and normal w_perp = w rotated
    // by +90 degrees; s'(i, j) and L(i, j) are affine in the pixel indices;
    // the half effective blur is hc = hc_fix + gR * L (eq. (17))
    double wx, wy, S00, L00, gR, hc_fix, lmax;
    if (G.beam == FP_PARALLEL) {
        // every ray runs along -u; s' = e.k - s_m, tau' = tau
        wx = -c;
        wy = -sn;
        S00 = sn * x0 - c * y0 - s;
        L00 = 0.0;
        gR = 0.0;
        hc_fix = 0.5 * G.tau;
        lmax = 0.0;
    } else {
        // the ray leaves the central ray (-u) at angle g towards e:
        // w = -cos g u + sin g e, e = (sn, -c)
        double cg, sg;
        if (G.beam == FP_FAN_ARC) {
            const double2 a = G.arc_cells[m + kBackPad];
            cg = a.x;
            sg = a.y;
            gR = (double)tab.ghr()[ray];                  // tan(tau / (2 D))
        } else {
            const double R = sqrt(D * D + s * s);
            cg = D / R;
            sg = s / R;
            gR = (double)tab.ghr()[ray] * R;              // g_m / 2
        }
        wx = -cg * c + sg * sn;
        wy = -cg * sn - sg * c;
        const double px = G.dsc * c, py = G.dsc * sn;
        S00 = -wy * (x0 - px) + wx * (y0 - py);
        L00 = wx * (x0 - px) + wy * (y0 - py);
        hc_fix = 0.0;
        // depth of the far side of the disk containing the image
        lmax = G.dsc * cg + G.half_diag;
    }
    const double wpx = -wy, wpy = wx;
    // March along the image axis closest to the ray; the other ("cross")
    // axis then advances s' by at least delta / sqrt(2) per pixel.  A wave
    // whose rays would march along different axes walks the union of both
    // row ranges with the wider window (the heaviest waves of a view, next
    // to the diagonal), so rays near a diagonal follow the axis of most of
    // their wave (its cross axis still advances s' by kFwdCrossMin delta
    // per pixel).  Every lane of the wave runs this (lanes past the last
    // cell walk the last ray).
    const double awx = fabs(wx), awy = fabs(wy);
    bool by_rows = awy >= awx;
    {
        const bool most = __popcll(__ballot(by_rows)) * 2 >= 64;
        if (fmin(awx, awy) >= kFwdAxisShare * fmax(awx, awy)) by_rows = most;
    }
    const int nq = by_rows ? G.nx : G.ny, nr = by_rows ? G.ny : G.nx;

    RayWalk<Real> w;
    const double zc = G.pixel * (by_rows ? wpx : wpy);
    const double zm = G.pixel * (by_rows ? wpy : wpx);
    const double lc = G.pixel * (by_rows ? wx : wy);
    const double lm = G.pixel * (by_rows ? wy : wx);
    w.trap.hab = tab.hab()[ray];
    w.trap.ia = tab.ia()[ray];
    w.trap.nhbia = tab.nhbia()[ray];
    w.trap.ha = tab.ha()[ray];
    w.dhq = (Real)(gR * lc);
    w.dhr = (Real)(gR * lm);
    w.zcr = (Real)zc;
    w.nq = nq;
    w.nr = nr;
    w.width = padded_width(G.nx, G.ny);
    w.row_stride = 2 * (size_t)w.width;
    w.img_stride = w.row_stride * (size_t)max(G.nx, G.ny);
    w.base = copies;
    // own copy: slot 0 (rows) or 1 (columns); the other copy the other slot
    // (read q of rotation k: by rows q = 0, 1, 2, 3 is k = 0, 3, 1, 2; by
    // columns k = 0, 1, 3, 2)
    {
        const int own = by_rows ? 0 : w.width, other = by_rows ? w.width : 0;
        w.qoff[0] = own;
        w.qoff[1] = other;
        w.qoff[2] = other;
        w.qoff[3] = own;
    }

    // Support |s'| < hab + hc, with hc bounded by its value at the far side
    // of the disk containing the image.
    const double hab_c = (double)w.trap.hab + hc_fix;
    const double izc = 1.0 / zc;
    const double hq = fma(gR, lmax, hab_c) * fabs(izc);   // half span along the cross axis
    // Rows whose window meets [0, nq): qf(r) = qf0 + r dq is the crossing.
    const double qf0 = -S00 * izc, dq = -zm * izc;
    const double q_lo_lim = -hq - 1.0, q_hi_lim = nq + hq;
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

    // The whole wave walks the union of its rays' rows, each block of rows
    // with one window width: control flow stays uniform, and rows or pixels
    // outside a ray's own range read the zero margin or evaluate to zero.
    int r0 = wave_min(r_lo);
    const int r1 = wave_max(r_hi);
    r0 = max(r0, 0);
    w.r0 = r0;
    w.hq = (float)hq * 1.000001f;   // (rounded up)
    // window start on row r: floor(-s'(0, r) / zc - hq) + 1
    w.X1 = 1.0 - (S00 + r0 * zm) * izc;
    w.dX = -zm * izc;
    w.hc0 = (Real)(hc_fix + gR * (L00 + r0 * lm));
    w.dhc = (Real)(gR * lm);
    // per-row half spans: hc = hc_fix + gR L, with L at most the depth where
    // the ray crosses the row, (L00 + qf0 lc) + r (dq lc + lm), plus the
    // window's half extent (hq + 1) |lc| (parallel beams: gR = 0, hq)
    {
        const double L0 = L00 + (qf0 + r0 * dq) * lc + (hq + 1.0) * fabs(lc) + r0 * lm;
        const double m = 1.0 + 1e-5;   // covers the FP32 rounding of the bound
        w.hqa = (float)(fma(gR, L0, hab_c) * fabs(izc) * m);
        w.hqb = (float)(gR * (dq * lc + lm) * fabs(izc) * m);
    }

    Real acc[NB * S];
#pragma unroll
    for (int k = 0; k < NB * S; ++k) acc[k] = 0;
    int nonzero = 0;
    if constexpr (kParts == 1) {
        if (r0 <= r1) walk_rows<Real, NB, MODE, S, TMAX>(w, r0, r1, acc, nonzero);
    } else {
        if (r0 <= r1) {
            // part p walks row blocks [p per, (p + 1) per)
            const int blocks = (r1 - r0) / kFwdBlockRows + 1;
            const int per = (blocks + kParts - 1) / kParts;
            const int ra = r0 + part * per * kFwdBlockRows;
            const int rb = min(r1, ra + per * kFwdBlockRows - 1);
            if (ra <= rb) walk_rows<Real, NB, MODE, S, TMAX>(w, ra, rb, acc, nonzero);
        }
        // the other parts hand their sums to part 0 through LDS (fixed
        // order: part 0's rows first)
        __shared__ Real part_acc[kParts - 1][NB * S][kRays];
        if (part > 0) {
#pragma unroll
            for (int k = 0; k < NB * S; ++k)
                part_acc[part - 1][k][threadIdx.x - part * kRays] = acc[k];
        }
        __syncthreads();
        if (part > 0) return;
#pragma unroll
        for (int q = 0; q < kParts - 1; ++q)
#pragma unroll
            for (int k = 0; k < NB * S; ++k) acc[k] += part_acc[q][k][threadIdx.x];
    }
    if (!active) return;
    const Real wbr = tab.wb()[ray];
    if constexpr (MODE == FwdMode::kCount) {
        counts[ray] = nonzero;
    } else if constexpr (MODE == FwdMode::kOnes) {
        const Real sum = acc[0] * wbr;
        out[ray] = sum != Real(0) ? Real(1) / sum : Real(0);
    } else {
#pragma unroll
        for (int k = 0; k < S; ++k) {
            // accumulator of rotation k (see above)
            const int q = S == 1 ? 0
                                 : (k == 0 ? 0 : k == 2 ? 3 : (k == 1) == by_rows ? 2 : 1);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                Real a = acc[b];
#pragma unroll
                for (int qq = 1; qq < S; ++qq)
                    if (q == qq) a = acc[qq * NB + b];
                const Real y = a * wbr;
                const size_t o = (size_t)(b * S + k) * nrays + ray;
                if constexpr (MODE == FwdMode::kPlain) {
                    out[o] = y;
                } else {  // kSirtResidual: row weights of the full view set
                    out[o] = row_w[(size_t)k * nrays + ray] * (y_meas[o] - y);
                }
            }
        }
    }
}

template <typename Real, int NB, FwdMode MODE, int S, int TMAX = (S == 1 ? 8 : 6)>
// (the quarter-turn walk of one image at 6 waves per SIMD, 80 VGPRs)
__global__ __launch_bounds__(kFwdThreads, S == 1 ? min_waves(NB, sizeof(Real)) : NB == 1 ? 6 : 1) void forward_kernel(
    DevGeom G, const Real *__restrict__ copies,
    Real *__restrict__ out, int *__restrict__ counts, const Real *__restrict__ y_meas,
    const Real *__restrict__ row_w) {
    forward_block<Real, NB, MODE, S, TMAX>(G, blockIdx.x, blockIdx.y, copies, out, counts, y_meas,
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
    Real gh[kPer], hab[kPer], ia[kPer], nhbia[kPer], ha[kPer], w[kPer][NB];
    int4 tc;   // tile entry of the view: M0, cnt, T, window constant (float bits)
};

// Two-component vector of the arithmetic type (float2 / double2).
template <typename Real>
struct Pair;
template <>
struct Pair<float> {
    using type = float2;
};
template <>
struct Pair<double> {
    using type = double2;
};

// Staged values of cell t as interleaved pairs, so that every value is read
// with an immediate offset from one base address: (blur, hab), (1/a,
// -(b-a)/(2a)), (a/2, weight of image 0), then the other images' weights two
// by two (an odd last one paired with zero); all scaled as the back tables.
// A weight is the sinogram value times the normalisation over the blur
// constant (table bwg).
constexpr int back_weight_pairs(int nb) { return nb / 2; }
static_assert(5 == kBackRayParams, "five per-ray parameters");
template <typename Real, int NB, int CAP>
struct BackLds {
    using P2 = typename Pair<Real>::type;
    P2 gh_hab[CAP], ia_nhbia[CAP], ha_w0[CAP];
    P2 w[back_weight_pairs(NB) > 0 ? back_weight_pairs(NB) : 1][CAP];
};
static_assert(sizeof(BackLds<float, 1, 64>) == back_lds_values(1) * 64 * sizeof(float),
              "back-projection staging size");

// Staged cell idx holds cell M0 - kBackPad + idx; the kBackPad cells on either
// side of [M0, M0 + cnt) get zero weight and harmless constants.  Image b
// reads sino + b nrays.  In the octant form (NB = 8, G.quarter_views = Q >
// 0, nrays = Q nd) images 4 + k read the reflected rays instead,
// ((Q - v + k Q) mod 4Q, nd-1-m), with weight zero for the views that are
// their own reflections (v = 0 and v = Q/2, the first and last of G).
template <typename Real, int NB, int CAP, BackMode MODE>
__device__ __forceinline__ void back_prefetch(const DevGeom &G, const RayTables<Real> &tab,
                                              const Real *__restrict__ sino, int v, int tile,
                                              int ntiles, size_t nrays,
                                              BackStage<Real, NB, CAP> &st) {
    st.tc = G.tile_cells[(size_t)v * ntiles + tile];
    const int M0 = st.tc.x, cnt = st.tc.y;
    const int n = cnt > 0 ? cnt + 2 * kBackPad : 0;
    // ray of the view's cell M0; byte offsets of rays fit 32 bits (fewer than
    // 2^30 rays), so each table is read from its uniform base plus one
    // per-lane offset
    const unsigned ray0 = (unsigned)v * (unsigned)G.nd + (unsigned)M0;
#pragma unroll
    for (int k = 0; k < BackStage<Real, NB, CAP>::kPer; ++k) {
        const int idx = (int)threadIdx.x + k * kBackThreads;
        if (idx < n) {
            // the padding cells repeat the constants of the nearest cell
            // (finite entries) with weight zero
            const int c = idx - kBackPad;
            const int cc = min(max(c, 0), cnt - 1);
            const unsigned off = (ray0 + (unsigned)cc) * (unsigned)sizeof(Real);
            auto at = [off](const Real *base) {
                return *reinterpret_cast<const Real *>(reinterpret_cast<const char *>(base) + off);
            };
            st.gh[k] = at(tab.bgh());
            st.hab[k] = at(tab.bhab());
            st.ia[k] = at(tab.bia());
            st.nhbia[k] = at(tab.nhbia());
            st.ha[k] = at(tab.bha());
            const Real wb = at(tab.bwg());
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                Real y;
                if constexpr (MODE == BackMode::kOnes) {
                    y = Real(1);
                } else if constexpr (NB == 8) {
                    const int Q = G.quarter_views;
                    if (b < 4 || Q == 0) {
                        y = at(sino + b * nrays);
                    } else if (v > 0 && v < G.nv - 1) {
                        const unsigned row = (unsigned)(Q - v + (b - 4) * Q);
                        y = sino[(size_t)row * G.nd + (unsigned)(G.nd - 1 - M0 - cc)];
                    } else {
                        y = Real(0);
                    }
                } else {
                    y = at(sino + b * nrays);
                }
                st.w[k][b] = c == cc ? y * wb : Real(0);
            }
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
            l.gh_hab[idx] = {st.gh[k], st.hab[k]};
            l.ia_nhbia[idx] = {st.ia[k], st.nhbia[k]};
            l.ha_w0[idx] = {st.ha[k], st.w[k][0]};
#pragma unroll
            for (int j = 0; j < back_weight_pairs(NB); ++j)
                l.w[j][idx] = {st.w[k][2 * j + 1], 2 * j + 2 < NB ? st.w[k][2 * j + 2] : Real(0)};
        }
    }
}

// part[k] += e * (weight of image k at staged cell idx); w0 is image 0's.
template <typename Real, int NB, int CAP>
__device__ __forceinline__ void back_accumulate(const BackLds<Real, NB, CAP> &l, int idx, Real e,
                                                Real w0, Real (&part)[NB]) {
    auto acc = [e](Real &p, Real w) { p = fma(e, w, p); };
    acc(part[0], w0);
#pragma unroll
    for (int j = 0; j < back_weight_pairs(NB); ++j) {
        const auto w = l.w[j][idx];
        constexpr int kLast = NB - 1;
        acc(part[2 * j + 1 <= kLast ? 2 * j + 1 : kLast], w.x);
        if (2 * j + 2 < NB)   // resolved at compile time (unrolled)
            acc(part[2 * j + 2 <= kLast ? 2 * j + 2 : kLast], w.y);
    }
}

// t times the cell spacing for t < kBackMaxUnrolled, held in scalar
// registers (the spacing is uniform)
template <typename Real>
struct CellSteps {
    Real v[kBackMaxUnrolled];
    __device__ explicit CellSteps(Real step) {
#pragma unroll
        for (int t = 0; t < kBackMaxUnrolled; ++t) v[t] = uniform((Real)t * step);
    }
    __device__ static float uniform(float x) {
        return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
    }
    __device__ static double uniform(double x) { return x; }
};

// Entries of one pixel with cells w0 .. w0 + T - 1 of the staged arrays
// (cell m = M0 - kBackPad + w0 + t).  num0 and ln0 are the numerators of s'
// and of R L at the first cell; cell t steps them by -t step hn and
// +t step hl.
template <typename Real, int NB, int CAP, bool UNROLLED>
__device__ __forceinline__ void back_window(const BackLds<Real, NB, CAP> &l, int w0, int T,
                                            const CellSteps<Real> &ts, Real stepr, Real num0,
                                            Real hn, Real ln0, Real hl, Real (&part)[NB]) {
    const auto *gh_hab = l.gh_hab + w0;
    const auto *ia_nhbia = l.ia_nhbia + w0;
    const auto *ha_w0 = l.ha_w0 + w0;
    // num = s' R_m and ln = R_m L at cell t; the staged constants carry R_m.
    // The entry is footprint / (ln g) times the weight; the staged weights
    // are already divided by the blur constant g, so only ln is inverted
    // (hc R_m = ln g then appears only inside the footprint's FMAs).
    auto entry = [&](int t, Real num, Real ln) {
        const auto a = gh_hab[t], b = ia_nhbia[t], c = ha_w0[t];
        const Real hcR = ln * a.x;
        const Trap<Real> p{a.y, b.x, b.y, c.x};
        const Real e = footprint_num(num, hcR, p) * fast_rcp(ln);
        back_accumulate<Real, NB, CAP>(l, w0 + t, e, c.y, part);
    };
    if constexpr (UNROLLED) {
        entry(0, num0, ln0);   // (an FMA by zero does not fold)
#pragma unroll
        for (int t = 1; t < kBackMaxUnrolled; ++t) {
            if (t >= T) break;  // T is uniform across the work-group
            entry(t, fma(-ts.v[t], hn, num0), fma(ts.v[t], hl, ln0));
        }
    } else {
        for (int t = 0; t < T; ++t) {
            const Real tstep = (Real)t * stepr;
            entry(t, fma(-tstep, hn, num0), fma(tstep, hl, ln0));
        }
    }
}

// Arc detector: entries of one pixel with cells w0 .. w0 + T - 1 of the
// staged arrays (cell m = m_first + t).  s' = rho sin(g_k - g_m) and
// L = rho cos(g_k - g_m), with rho and g_k the distance and angle of the
// pixel centre from the source.  Unrolled: a0 and b0 are s' and L at the
// first cell, and cell t is their rotation by t times the angular pitch.
// Wide windows: s' = cos g_m (e.k) - sin g_m h and L = cos g_m h + sin g_m (e.k)
// per cell in FP64.
template <typename Real, int NB, int CAP, bool UNROLLED>
__device__ __forceinline__ void back_window_arc(const BackLds<Real, NB, CAP> &l, const DevGeom &G,
                                                int w0, int T, int m_first, double ek, double h,
                                                Real (&part)[NB]) {
    const auto *gh_hab = l.gh_hab + w0;
    const auto *ia_nhbia = l.ia_nhbia + w0;
    const auto *ha_w0 = l.ha_w0 + w0;
    // (staged weights divided by the blur constant, as in back_window)
    auto entry = [&](int t, Real sp, Real L) {
        const auto a = gh_hab[t], b = ia_nhbia[t], c = ha_w0[t];
        const Real hc = L * a.x;
        const Trap<Real> p{a.y, b.x, b.y, c.x};
        const Real e = footprint_num(sp, hc, p) * fast_rcp(L);
        back_accumulate<Real, NB, CAP>(l, w0 + t, e, c.y, part);
    };
    const double2 *cells = G.arc_cells + m_first + kBackPad;
    if constexpr (UNROLLED) {
        const double2 g = cells[0];
        const Real a0 = (Real)(g.x * ek - g.y * h);
        const Real b0 = (Real)(g.x * h + g.y * ek);
        entry(0, a0, b0);
#pragma unroll
        for (int t = 1; t < kBackMaxUnrolled; ++t) {
            if (t >= T) break;  // T is uniform across the work-group
            Real rc, rs;
            arc_rotation<Real>(G, t, rc, rs);
            entry(t, fma(-b0, rs, a0 * rc), fma(a0, rs, b0 * rc));
        }
    } else {
        for (int t = 0; t < T; ++t) {
            const double2 g = cells[t];
            entry(t, (Real)(g.x * ek - g.y * h), (Real)(g.x * h + g.y * ek));
        }
    }
}

// One tile (tx, ty) and view group `group` of `groups`.
template <typename Real, int NB, int CAP, BackMode MODE, int BEAM>
__device__ __forceinline__ void back_block(BackLds<Real, NB, CAP> (&lds)[2], const DevGeom &G,
                                           int tx, int ty, int group, int groups,
                                           bool to_partial,
                                           const Real *__restrict__ sino, Real *__restrict__ img,
                                           Real *__restrict__ partial,
                                           const Real *__restrict__ col_w, Real relaxation) {
    const RayTables<Real> &tab = ray_tables<Real>(G);

    const int tile = ty * G.tiles_x + tx;
    const int ntiles = G.tiles_x * G.tiles_y;
    const size_t npix = (size_t)G.nx * G.ny;
    // sinogram values between the images of the batch (octant form: between
    // the quarter turns of the one image)
    const size_t nrays = (size_t)(G.quarter_views > 0 ? G.quarter_views : G.nv) * G.nd;
    const int v_begin = (int)(((long)G.nv * group) / groups);
    const int v_end = (int)(((long)G.nv * (group + 1)) / groups);
    constexpr int P = kBackPixPerThread;
    constexpr int kRowStep = kBackThreads / kBackTileW;
    // A wave covers 16 columns x 4 rows of the tile, and each quarter-wave
    // (16 lanes, served together by the LDS) a 4 x 4 block of them, whose
    // windows lie within a few cells of each other: fewer LDS bank conflicts
    // than a 16 x 1 row, whose windows spread over up to ~24 cells.
    static_assert(kBackTileW == 16 && kBackThreads == 256, "lane -> pixel map");
    const unsigned t = threadIdx.x;
    const int i = tx * kBackTileW + (int)((t & 3u) | (((t >> 4) & 3u) << 2));
    const int j0 = ty * kBackTileH + (int)(((t >> 2) & 3u) | ((t >> 6) << 2));
    bool valid[P];
#pragma unroll
    for (int p = 0; p < P; ++p) valid[p] = i < G.nx && j0 + p * kRowStep < G.ny;
    const double xk = (i - 0.5 * (G.nx - 1)) * G.pixel;
    const double yk0 = (j0 - 0.5 * (G.ny - 1)) * G.pixel;
    const double ystep = kRowStep * G.pixel;
    const double D = G.dsd, step = G.cell_step, c0 = 0.5 * (G.nd - 1);
    const Real Dr = (Real)D, stepr = (Real)step;
    const float istep = (float)(1.0 / step);
    const float Distep = (float)(D / step);
    const CellSteps<Real> tsteps(stepr);

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
            const float wc = __int_as_float(tc.w);
            // (buffer offset formed in scalar registers: v is uniform)
            const BackLds<Real, NB, CAP> &l = *reinterpret_cast<const BackLds<Real, NB, CAP> *>(
                reinterpret_cast<const char *>(&lds[0]) +
                __builtin_amdgcn_readfirstlane((v & 1) * (int)sizeof(BackLds<Real, NB, CAP>)));
            if (v + 1 < v_end)
                back_prefetch<Real, NB, CAP, MODE>(G, tab, sino, v + 1, tile, ntiles, nrays, st);

            if (cnt > 0) {
                const double2 cs = G.views[v];
                double ek = xk * cs.y - yk0 * cs.x;             // e . k
                double h = G.dsc - (xk * cs.x + yk0 * cs.y);    // D_sc - u . k
                const double dek = -ystep * cs.x, dh = -ystep * cs.y;
                // Window start in staged cells: w0 = m_lo - (M0 - kBackPad) with
                // m_lo = floor((c_k - H) / step + c0) + 1, H the tile's bound on
                // |c_k - c_m| over non-zero cells (the first cell past
                // c_k - H), clamped to the staged range; the tile table folds
                // the constants into wc, so per pixel it is the integer part
                // of c_k / step + wc clamped to [0, w_hi].
                const int base = M0 - kBackPad;
                // coordinate of staged cell 0
                const double s_base = ((double)base - c0) * step;
                const int w_hi = cnt + 2 * kBackPad - min(T, cnt + 2 * kBackPad);
                const float w_hif = (float)w_hi;
                const int Tw = T <= kBackMaxUnrolled ? T : min(T, cnt + 2 * kBackPad);
#pragma unroll
                for (int p = 0; p < P; ++p, ek += dek, h += dh) {
                    // the pixel's coordinate c_k (flat: its shadow
                    // s_k = D (e.k) / h; parallel: e.k; arc: its angle
                    // atan(e.k / h)); the window never passes a non-zero
                    // cell
                    const float hf = (float)h, ekf = (float)ek;
                    float wf;
                    if constexpr (BEAM == FP_PARALLEL)
                        wf = fmaf(ekf, istep, wc);
                    else if constexpr (BEAM == FP_FAN_ARC)
                        wf = fmaf(atanf(ekf * fast_rcp(hf)), istep, wc);
                    else
                        wf = fmaf(Distep * ekf, fast_rcp(hf), wc);
                    const int w0 = (int)__builtin_amdgcn_fmed3f(wf, 0.0f, w_hif);
                    if constexpr (BEAM == FP_FAN_ARC) {
                        if (T <= kBackMaxUnrolled)
                            back_window_arc<Real, NB, CAP, true>(l, G, w0, Tw, base + w0, ek, h,
                                                                 blk[p]);
                        else
                            back_window_arc<Real, NB, CAP, false>(l, G, w0, Tw, base + w0, ek,
                                                                  h, blk[p]);
                    } else {
                        // s' = num / R_m and R_m L = ln with
                        // num = D (e.k) - s_m h, ln = D h + s_m (e.k)
                        // (parallel: num = e.k - s_m, ln = 1), at the
                        // window's first cell in FP64, then steps of one cell
                        const double s_first = fma((double)w0, step, s_base);
                        Real num0, hn, ln0, hl;
                        if constexpr (BEAM == FP_PARALLEL) {
                            num0 = (Real)(ek - s_first);
                            hn = Real(1);
                            ln0 = Real(1);
                            hl = Real(0);
                        } else {
                            num0 = (Real)(D * ek - s_first * h);
                            hn = (Real)h;
                            hl = (Real)ek;
                            ln0 = fma((Real)s_first, hl, Dr * hn);
                        }
                        if (T <= kBackMaxUnrolled)
                            back_window<Real, NB, CAP, true>(l, w0, Tw, tsteps, stepr, num0, hn,
                                                             ln0, hl, blk[p]);
                        else
                            back_window<Real, NB, CAP, false>(l, w0, Tw, tsteps, stepr, num0, hn,
                                                              ln0, hl, blk[p]);
                    }
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
        if (to_partial) {
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

// to_partial: write the per-group sums to `partial` ([group][NB][npix]) even
// with one group (the quarter-turn form combines them in its own finalize).
template <typename Real, int NB, int CAP, BackMode MODE, int BEAM>
__global__ __launch_bounds__(kBackThreads, min_waves(NB, sizeof(Real))) void back_kernel(
    DevGeom G, const Real *__restrict__ sino, Real *__restrict__ img, Real *__restrict__ partial,
    const Real *__restrict__ col_w, Real relaxation, int to_partial) {
    __shared__ BackLds<Real, NB, CAP> lds[2];
    // One work-group per (tile, view group), n = tiles x groups of them in a
    // 1-D grid, group-major.  Work-group L runs on XCD L mod kXcds.  With one
    // view group the XCDs take contiguous ranges of tiles, so each works on
    // one band of neighbouring tiles, whose cells are a fraction of the
    // detector in every view, and its L2 streams only those cells' per-ray
    // tables (3 % less back time at 1024^2 and 2048^2).  With several groups
    // (small images) that remapping measured slower, and work-group L takes
    // item L.
    const unsigned ntiles = (unsigned)(G.tiles_x * G.tiles_y), n = gridDim.x;
    const unsigned groups = n / ntiles, L = blockIdx.x;
    unsigned P = L;
    if (groups == 1) {
        const unsigned k = L % kXcds, per = n / kXcds, extra = n % kXcds;
        P = k * per + min(k, extra) + L / kXcds;
    }
    const int tile = (int)(P % ntiles), group = (int)(P / ntiles);
    back_block<Real, NB, CAP, MODE, BEAM>(lds, G, tile % G.tiles_x, tile / G.tiles_x, group,
                                          (int)groups, groups > 1 || to_partial != 0, sino, img,
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

// Quarter-turn form of the back projection: the back kernel ran over the
// first quarter of the views with the sinogram rows of view v + k nv as
// image k (k < 4) of each input image, so its sum for image k at pixel p is
// the contribution of views v + k nv at pixel R^k p (R(i, j) = (n-1-j, i);
// the entries of view v + k nv at R^k p equal those of view v at p).  Pixel
// (i, j) of the result is therefore
//   sum_g [P_0(i, j) + P_1(j, n-1-i) + P_2(n-1-i, n-1-j) + P_3(n-1-j, i)],
// P_k(a, b) the group-g partial of image k at column a, row b.  Block
// (32, 32) finishes a 32 x 32 tile of image blockIdx.z, one pixel per
// thread; the two transposed terms go through LDS so that every global
// access is coalesced.  Sums are taken in a fixed order (groups inside,
// rotations outside).
template <BackMode MODE>
__device__ __forceinline__ void finalize_quarter_tile(const float *__restrict__ partial,
                                                      int groups, int nb4, int n, int im, int i0,
                                                      int j0, float *__restrict__ img,
                                                      const float *__restrict__ col_w,
                                                      float relaxation) {
    __shared__ float t1[32][33], t3[32][33];
    const size_t npix = (size_t)n * n;
    const int tx = threadIdx.x, ty = threadIdx.y;
    auto part = [&](int g, int k) { return partial + ((size_t)g * nb4 + im * 4 + k) * npix; };
    // t1[a][b] = P_1(j0 + b, n-1-i0-a), t3[a][b] = P_3(n-1-j0-b, i0 + a), with
    // a = ty, b = tx (reads along b)
    {
        float s1 = 0.0f, s3 = 0.0f;
        if (i0 + ty < n && j0 + tx < n) {
            for (int g = 0; g < groups; ++g) {
                s1 += part(g, 1)[(size_t)(n - 1 - i0 - ty) * n + (j0 + tx)];
                s3 += part(g, 3)[(size_t)(i0 + ty) * n + (n - 1 - j0 - tx)];
            }
        }
        t1[ty][tx] = s1;
        t3[ty][tx] = s3;
    }
    __syncthreads();
    const int i = i0 + tx, j = j0 + ty;
    if (i >= n || j >= n) return;
    float z0 = 0.0f, z2 = 0.0f;
    for (int g = 0; g < groups; ++g) {
        z0 += part(g, 0)[(size_t)j * n + i];
        z2 += part(g, 2)[(size_t)(n - 1 - j) * n + (n - 1 - i)];
    }
    const float z = ((z0 + t1[tx][ty]) + z2) + t3[tx][ty];
    const size_t pix = (size_t)j * n + i;
    if constexpr (MODE == BackMode::kPlain) {
        img[(size_t)im * npix + pix] = z;
    } else {  // kSirtUpdate
        img[(size_t)im * npix + pix] += relaxation * col_w[pix] * z;
    }
}

template <BackMode MODE>
__global__ __launch_bounds__(1024) void back_finalize_quarter_kernel(
    const float *__restrict__ partial, int groups, int nb4, int n, float *__restrict__ img,
    const float *__restrict__ col_w, float relaxation) {
    finalize_quarter_tile<MODE>(partial, groups, nb4, n, blockIdx.z, blockIdx.x * 32,
                                blockIdx.y * 32, img, col_w, relaxation);
}

// Octant form of the back projection (one image): the back kernel ran over
// the base views v = 0 .. Q/2 with the sinogram rows v + k Q as image k and
// the reflected rays ((Q - v + k Q) mod 4Q, nd-1-m) as image 4 + k (k < 4),
// so its sum for image k at pixel p is the contribution of views v + k Q at
// R^k p, and for image 4 + k that of the reflected views at R^k D p
// (D(i, j) = (j, i)).  Pixel q = (i, j) of the result is therefore
//   sum_g sum_k [P_k(R^-k q) + M_k(D R^-k q)]
//   = sum_g [P_0(i, j) + P_1(j, n-1-i) + P_2(n-1-i, n-1-j) + P_3(n-1-j, i)
//          + M_0(j, i) + M_1(n-1-i, j) + M_2(n-1-j, n-1-i) + M_3(i, n-1-j)],
// P_k = image k and M_k = image 4 + k of the group-g partials, at (column,
// row).  Block (32, 32) finishes a 32 x 32 tile, one pixel per thread; the
// four terms with swapped coordinates go through LDS so that every global
// access is coalesced.  Sums in a fixed order.
template <BackMode MODE>
__global__ __launch_bounds__(1024) void back_finalize_octant_kernel(
    const float *__restrict__ partial, int groups, int n, float *__restrict__ img,
    const float *__restrict__ col_w, float relaxation) {
    __shared__ float t[4][32][33];
    const size_t npix = (size_t)n * n;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    auto part = [&](int g, int k) { return partial + ((size_t)g * 8 + k) * npix; };
    // t[.][a][b], a = ty, b = tx (reads along b): P_1(j0 + b, n-1-i0-a),
    // P_3(n-1-j0-b, i0 + a), M_0(j0 + b, i0 + a), M_2(n-1-j0-b, n-1-i0-a)
    {
        float s1 = 0.0f, s3 = 0.0f, s4 = 0.0f, s6 = 0.0f;
        if (i0 + ty < n && j0 + tx < n) {
            const size_t ra = (size_t)(n - 1 - i0 - ty) * n, rb = (size_t)(i0 + ty) * n;
            const int ca = j0 + tx, cb = n - 1 - j0 - tx;
            for (int g = 0; g < groups; ++g) {
                s1 += part(g, 1)[ra + ca];
                s3 += part(g, 3)[rb + cb];
                s4 += part(g, 4)[rb + ca];
                s6 += part(g, 6)[ra + cb];
            }
        }
        t[0][ty][tx] = s1;
        t[1][ty][tx] = s3;
        t[2][ty][tx] = s4;
        t[3][ty][tx] = s6;
    }
    __syncthreads();
    const int i = i0 + tx, j = j0 + ty;
    if (i >= n || j >= n) return;
    float z0 = 0.0f, z2 = 0.0f, z5 = 0.0f, z7 = 0.0f;
    for (int g = 0; g < groups; ++g) {
        z0 += part(g, 0)[(size_t)j * n + i];
        z2 += part(g, 2)[(size_t)(n - 1 - j) * n + (n - 1 - i)];
        z5 += part(g, 5)[(size_t)j * n + (n - 1 - i)];
        z7 += part(g, 7)[(size_t)(n - 1 - j) * n + i];
    }
    const float zr = ((z0 + t[0][tx][ty]) + z2) + t[1][tx][ty];
    const float zm = ((t[2][tx][ty] + z5) + t[3][tx][ty]) + z7;
    const float z = zr + zm;
    const size_t pix = (size_t)j * n + i;
    if constexpr (MODE == BackMode::kPlain) {
        img[pix] = z;
    } else {  // kSirtUpdate
        img[pix] += relaxation * col_w[pix] * z;
    }
}

}  // namespace
}  // namespace fanproj
