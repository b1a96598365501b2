// Device kernels of the patop library (gfx950).
//
// Forward A (Alg. 1):
//   1. k_fill            f <- 0  (FP64 fine-bin coefficients, [B][K][Mcount])
//   2. k_fwd_wave /      closed form: one work-group of one wave per (4 x 4 x 4
//      k_fwd_quad        voxel cube, chunk of transducers): for each transducer,
//                        every voxel of the cube adds p0 * |M_i^m| (Alg. 3, Eq.
//                        ui_area) into an LDS FP64 histogram covering the cube's
//                        bin window, which the wave then adds to f with FP64
//                        atomics, with no work-group barrier.  Quadrature: one
//                        256-thread work-group per (voxel brick, chunk), p0 * dA / r
//                        into the bin of each surface point (Alg. 2, Eq.
//                        def_f_point).  Sparse forward: k_support_count / _scan /
//                        _write list the voxels that are nonzero in some volume,
//                        and k_fwd_sparse_wave strides waves of 64 of them.  Time
//                        tiles: k_fwd_tile owns a (transducer, tile) of f.
//   3. k_fir             s_hat[l] = sum_j G[j] scale[m] f[m], m = U l - j (FP64): the
//                        convolution with h followed by the block average D_U
//                        (Eq. discrete_conv, Eq. def_downsampling) as one
//                        polyphase filter G[j] = 1/U sum_{l'=1..U} h[j + l'];
//                        scale[m] = U fs dr^2 / (c tau_{m-1/2}) (surface, Eq.
//                        ui_area) or U fs dr (points).
// Adjoint A^T (Alg. 5-7):
//   1. k_adjw            W[m] = scale[m] sum_l G[U l - m] y[l]: transpose of the
//                        block average and correlation with the reversed kernel.
//   2. k_adj_wave /      one work-group per (cube of one wave, or brick for the
//      k_adj_quad        quadrature, chunk of transducers): W of the bin window is
//                        staged in LDS, every voxel gathers sum_m |M_i^m| W[m]
//                        (FP32 or FP64 per transducer) and accumulates over
//                        transducers in FP64.
//   3. k_finish          cast of the FP64 sums when transducer chunks were split
//                        over work-groups.
#include <hip/hip_runtime.h>

#include "area.h"
#include "kernels.h"

namespace patop {

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------

__global__ void k_fill(double* __restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

template <class Real>
__global__ void k_finish(const double* __restrict__ z, Real* __restrict__ out, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (Real)z[i];
}

__device__ __forceinline__ int floordiv(int a, int b)
{
    int q = a / b;
    return (q * b > a) ? q - 1 : q;
}

// the voxel owned by this thread and the box of the work-group's brick
struct Brick {
    int64_t idx;
    int ix, iy, iz;
    bool valid;
    double lo[3], hi[3];   // axis-aligned box of the brick's voxel centres (global)
};

// axis-aligned box of brick bid's voxel centres (global coordinates)
__device__ __forceinline__ void brick_box(const KParams& P, int bid, double lo[3], double hi[3])
{
    const int bxi = bid % P.nbx, byi = (bid / P.nbx) % P.nby, bzi = bid / (P.nbx * P.nby);
    const int x0 = bxi * kBrickX, y0 = byi * kBrickY, z0 = bzi * kBrickZ;
    const int x1 = (int)min((int64_t)(x0 + kBrickX), P.n[0]) - 1;
    const int y1 = (int)min((int64_t)(y0 + kBrickY), P.n[1]) - 1;
    const int z1 = (int)min((int64_t)(z0 + kBrickZ), P.n[2]) - 1;
    lo[0] = P.origin[0] + x0 * P.w; hi[0] = P.origin[0] + x1 * P.w;
    lo[1] = P.origin[1] + y0 * P.w; hi[1] = P.origin[1] + y1 * P.w;
    lo[2] = P.origin[2] + z0 * P.w; hi[2] = P.origin[2] + z1 * P.w;
}

__device__ __forceinline__ void brick_setup(const KParams& P, int bid, Brick& Bk)
{
    const int bxi = bid % P.nbx, byi = (bid / P.nbx) % P.nby, bzi = bid / (P.nbx * P.nby);
    const int x0 = bxi * kBrickX, y0 = byi * kBrickY, z0 = bzi * kBrickZ;
    // each wave owns a 4 x 4 x 4 sub-cube of the brick: the most compact set of
    // 64 voxels, so that their sweeps over a transducer have similar lengths
    // and quadrant counts (less divergence than an 8 x 8 x 1 slab)
    const int v = threadIdx.x, w = v >> 6, l = v & 63;
    Bk.ix = x0 + (w & 1) * 4 + (l & 3);
    Bk.iy = y0 + (w >> 1) * 4 + ((l >> 2) & 3);
    Bk.iz = z0 + (l >> 4);
    Bk.valid = Bk.ix < P.n[0] && Bk.iy < P.n[1] && Bk.iz < P.n[2];
    Bk.idx = Bk.valid ? Bk.ix + P.n[0] * (Bk.iy + P.n[1] * (int64_t)Bk.iz) : 0;
    brick_box(P, bid, Bk.lo, Bk.hi);
}

// shells that any voxel of the box [lo, hi] can reach on transducer T
// (bounding sphere; Eq. rmin_rmax bounds each pair's range inside it), clipped
// to the kept shells [Jlo, Jhi]: empty (wlo > whi) if none
__device__ __forceinline__ void box_window(const KParams& P, const double lo3[3], const double hi3[3],
                                           const TrDev& T, int& wlo, int& whi)
{
    double dd = 0.0, dm = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double o = fmax(0.0, fmax(lo3[a] - T.cen[a], T.cen[a] - hi3[a]));
        dd += o * o;
        double f = fmax(fabs(lo3[a] - T.cen[a]), fabs(hi3[a] - T.cen[a]));
        dm += f * f;
    }
    double dlo = fmax(sqrt(dd) - T.rad, 0.0), dhi = sqrt(dm) + T.rad;
    int64_t lo = (int64_t)floor(dlo - P.r0);
    int64_t hi = (int64_t)ceil(dhi - P.r0) + 1;
    lo = max(lo, P.Jlo);
    hi = min(hi, P.Jhi);
    wlo = (int)lo;
    whi = (int)hi;
}

__device__ __forceinline__ void brick_window(const KParams& P, const Brick& Bk, const TrDev& T, int& wlo,
                                             int& whi)
{
    box_window(P, Bk.lo, Bk.hi, T, wlo, whi);
}

// shells that the voxel at frame coordinates x can reach on transducer T: from
// its distances to the nearest and the farthest point of the surface (Eq.
// rmin_rmax), in closed form.  Planar: the rectangle's nearest and farthest
// points in its plane.  Cylinder: |x - y|^2 = R^2 + rho^2 - 2 R rho cos(delta)
// + (z - x3)^2 for the point y at angle gap delta from the voxel's direction,
// whose smallest gap is 0 inside the angular range and |theta_i| - theta_max
// outside it, and largest min(pi, |theta_i| + theta_max); rho cos(delta) from
// the frame coordinates and cos / sin of theta_max, with no angle computed.
// floor / ceil keep a shell of margin for rounding: [lo, hi] holds every bin of
// every quadrant sweep of the pair.
__device__ __forceinline__ void pair_range(const TrDev& T, const double x[3], double r0, int& lo, int& hi)
{
    double dmin2, dmax2;
    if (T.shape == 0) {
        const double du = fmax(0.0, fabs(x[0]) - T.p[0]), dv = fmax(0.0, fabs(x[1]) - T.p[1]);
        const double eu = fabs(x[0]) + T.p[0], ev = fabs(x[1]) + T.p[1];
        const double z2 = x[2] * x[2];
        dmin2 = fma(du, du, fma(dv, dv, z2));
        dmax2 = fma(eu, eu, fma(ev, ev, z2));
    } else {
        const double R = T.p[0], ax1 = fabs(x[1]);
        const double rho2 = fma(x[0], x[0], x[1] * x[1]);
        const double rho = sqrt(rho2);
        const bool inside = fma(x[0], T.sth, -ax1 * T.cth) >= 0.0;   // |theta_i| <= theta_max
        const double cmin = inside ? rho : fma(x[0], T.cth, ax1 * T.sth);
        const double cmax = x[0] < -T.cth * rho ? -rho : fma(x[0], T.cth, -ax1 * T.sth);
        const double vmin = fmax(0.0, fabs(x[2]) - T.p[2]), vmax = fabs(x[2]) + T.p[2];
        const double base = fma(R, R, rho2);
        dmin2 = fma(vmin, vmin, fma(-2.0 * R, cmin, base));
        dmax2 = fma(vmax, vmax, fma(-2.0 * R, cmax, base));
    }
    lo = (int)floor(sqrt(fmax(dmin2, 0.0)) - r0);
    hi = (int)ceil(sqrt(fmax(dmax2, 0.0)) - r0) + 1;
}

// [min lo, max hi] over the lanes of the wave that take part (others pass
// INT_MAX / INT_MIN), clipped to the kept shells [Jlo, Jhi]
__device__ __forceinline__ void wave_window(const KParams& P, int lo, int hi, int& wlo, int& whi)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
    }
    wlo = (int)max((int64_t)lo, P.Jlo);
    whi = (int)min((int64_t)hi, P.Jhi);
}

// frame coordinates of a voxel (Sec. 4.1 / Sec. 4.2 frames), FP64
__device__ __forceinline__ void frame_coords(const TrDev& T, int ix, int iy, int iz, double x[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = fma(T.g[a][0], ix, fma(T.g[a][1], iy, fma(T.g[a][2], iz, T.base[a])));
}

// ---------------------------------------------------------------------------
// per-pair geometry: reflected quadrants of the parameter rectangle
// (Eq. uvminmax; Eq. folded_intervals for the cylinder), built one at a time
// ---------------------------------------------------------------------------

// Two reflected intervals that share an end point, [e, p] and [e, q] (or [p, e]
// and [q, e]), cover the same parameter region as the interval between e and
// the nearer of p, q counted twice plus the remainder counted once.  Sweeping
// the merged form visits each bin of the shared part once instead of twice.
struct WInt {
    double lo[2], hi[2];
    float w[2];
    int n;
};

// intervals [0, A] and [0, B] (A, B >= 0), Eq. uvminmax with the origin inside.
// MERGE: the shared-part form above; else the two intervals as they are, which
// an approximation that is not additive over sub-intervals (the trapezoidal
// I_l: the chord of a split arc is not the chord of the arc) must use.
template <bool MERGE = true>
__device__ __forceinline__ void split_at_zero(double A, double B, WInt& I)
{
    if (MERGE) {
        double m = fmin(A, B), M = fmax(A, B);
        I.lo[0] = 0.0; I.hi[0] = m; I.w[0] = 2.0f;
        I.lo[1] = m;   I.hi[1] = M; I.w[1] = 1.0f;
    } else {
        I.lo[0] = 0.0; I.hi[0] = A; I.w[0] = 1.0f;
        I.lo[1] = 0.0; I.hi[1] = B; I.w[1] = 1.0f;
    }
    I.n = 2;
}

// the reflected intervals of [lo, hi] about 0 (Eq. uvminmax)
template <bool MERGE = true>
__device__ __forceinline__ void fold_line(double lo, double hi, WInt& I)
{
    if (lo < 0.0 && 0.0 < hi) { split_at_zero<MERGE>(-lo, hi, I); return; }
    double a = fabs(lo), b = fabs(hi);
    I.lo[0] = fmin(a, b); I.hi[0] = fmax(a, b); I.w[0] = 1.0f;
    I.lo[1] = I.hi[1] = 0.0; I.w[1] = 0.0f;
    I.n = 1;
}

template <class AT>
struct PlanarPair {
    WInt U, V;
    double z2;
    __device__ __forceinline__ void bind(double*, const double2*) {}
    __device__ __forceinline__ void setup(const TrDev& T, const double x[3], double)
    {
        double L1 = T.p[0], L2 = T.p[1];
        fold_line(-L1 - x[0], L1 - x[0], U);
        fold_line(-L2 - x[1], L2 - x[1], V);
        z2 = x[2] * x[2];
    }
    // bins wlo .. whi of each quadrant reach the sink (each quadrant is walked
    // from its first bin, see pl_sweep)
    template <class Sink>
    __device__ __forceinline__ void sweep(int wlo, int whi, Sink& sink, double r0)
    {
        // the lane's non-empty quadrants first, so lanes step through their k-th
        // quadrant together
        int list = 0, nq = 0;
#pragma unroll
        for (int qi = 0; qi < 4; ++qi) {
            const int i = qi >> 1, j = qi & 1;
            const bool ok = i < U.n && j < V.n && (i ? U.hi[1] > U.lo[1] : U.hi[0] > U.lo[0]) &&
                            (j ? V.hi[1] > V.lo[1] : V.hi[0] > V.lo[0]);
            if (ok) { list |= qi << (2 * nq); ++nq; }
        }
#pragma unroll 1
        for (int t = 0; t < nq; ++t) {
            const int qi = (list >> (2 * t)) & 3;
            const int i = qi >> 1, j = qi & 1;
            const double a = i ? U.lo[1] : U.lo[0], b = i ? U.hi[1] : U.hi[0];
            const double c = j ? V.lo[1] : V.lo[0], d = j ? V.hi[1] : V.hi[0];
            const float w = (i ? U.w[1] : U.w[0]) * (j ? V.w[1] : V.w[0]);
            PlQuad<AT> q;
            pl_setup(q, a, b, c, d, z2, r0);
            pl_sweep(q, wlo, whi, (AT)w, sink);
        }
    }
};

__device__ __forceinline__ double wrap_pi(double u)
{
    if (u <= -M_PI) u += 2.0 * M_PI;
    if (u <= -M_PI) u += 2.0 * M_PI;
    if (u > M_PI) u -= 2.0 * M_PI;
    if (u > M_PI) u -= 2.0 * M_PI;
    return u;
}

// The interval ends of the folded quadrants live in LDS (one column per thread,
// kBoxSlots doubles), read back per quadrant: kept in registers they would be
// live through every sweep and pushed to scratch memory at three or four waves
// per SIMD.
constexpr int kBoxSlots = 8;

// MERGE of the folded intervals holds for every I_l that is a difference of a
// function of the end points (exact, tables); not for the chord.
template <int NW, int IL, int STRIDE = kThreads>   // STRIDE: threads of the work-group (the table's row)
struct CylinderPair {
    static constexpr bool kMerge = IL != kIlTrapezoid;
    CyPair P;
    double* box;             // this thread's column of the LDS box table
    int list, nq;            // non-empty quadrants (2 bits each, in sweep order) and their number
    int wbits;               // quadrant weights: bits 0/1 the U intervals, 2/3 the V intervals (set = 2)
    __device__ __forceinline__ void bind(double* table, const double2* lut)
    {
        box = table + threadIdx.x;
        P.lut = lut;
    }
    __device__ __forceinline__ void setup(const TrDev& T, const double x[3], double)
    {
        WInt U, V;
        double R = T.p[0], th = T.p[1], Lz = T.p[2];
        // a voxel on the focal line (rho = 0, Sec. 4.2) has no angular position;
        // rounding of its frame coordinates leaves rho at ~1e-16 of them, which
        // is snapped to 0 so that its angle is 0 rather than an arbitrary one
        double rho = sqrt64(x[0] * x[0] + x[1] * x[1]);
        if (rho <= 1e-10 * R) rho = 0.0;
        double thi = (rho > 0.0) ? atan2_full(x[1], x[0]) : 0.0;
        P.R = R;
        P.dm = fabs(R - rho);
        P.mu = 4.0 * R * rho;
        P.imu = P.mu > 0.0 ? rcp64_full(P.mu) : 0.0;
        double u1 = wrap_pi(-th - thi), u2 = wrap_pi(th - thi);
        // Eq. folded_intervals (merged where the areas are exact, see split_at_zero)
        if (u1 < 0.0 && 0.0 < u2) {
            split_at_zero<kMerge>(-u1, u2, U);
        } else if (u2 < u1) {
            // [u1, pi] and [-u2, pi]
            if (!kMerge) {
                U.lo[0] = u1;  U.hi[0] = M_PI; U.w[0] = 1.0f;
                U.lo[1] = -u2; U.hi[1] = M_PI; U.w[1] = 1.0f;
            } else {
                double m = fmax(u1, -u2), M = fmin(u1, -u2);
                U.lo[0] = m; U.hi[0] = M_PI; U.w[0] = 2.0f;
                U.lo[1] = M; U.hi[1] = m;    U.w[1] = 1.0f;
            }
            U.n = 2;
        } else if (0.0 <= u1) {
            U.lo[0] = u1; U.hi[0] = u2; U.w[0] = 1.0f; U.n = 1;
        } else {
            U.lo[0] = -u2; U.hi[0] = -u1; U.w[0] = 1.0f; U.n = 1;
        }
        fold_line<kMerge>(-Lz - x[2], Lz - x[2], V);
        // the non-empty quadrants in decreasing order of their number of bins
        // (nearest to farthest corner, estimated in FP32): the wave steps
        // through every lane's t-th quadrant together, so the lanes' longest
        // sweeps share one trip count
        bool ok[4];
        float len[4];
        {
            const float muf = (float)P.mu, dm2 = (float)(P.dm * P.dm);
            float pa[2], pb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const float sa = __sinf(0.5f * (float)(i < U.n ? U.lo[i] : 0.0));
                const float sb = __sinf(0.5f * (float)(i < U.n ? U.hi[i] : 0.0));
                pa[i] = fmaf(muf * sa, sa, dm2);
                pb[i] = fmaf(muf * sb, sb, dm2);
            }
#pragma unroll
            for (int qi = 0; qi < 4; ++qi) {
                const int i = qi >> 1, j = qi & 1;
                ok[qi] = i < U.n && j < V.n && (i ? U.hi[1] > U.lo[1] : U.hi[0] > U.lo[0]) &&
                         (j ? V.hi[1] > V.lo[1] : V.hi[0] > V.lo[0]);
                const float c = (float)(j < V.n ? V.lo[j] : 0.0), d = (float)(j < V.n ? V.hi[j] : 0.0);
                len[qi] = ok[qi] ? fmaxf(sqrt_t(fmaf(d, d, pb[i])) - sqrt_t(fmaf(c, c, pa[i])), 0.0f) : -1.0f;
            }
        }
        list = 0;
        nq = 0;
#pragma unroll
        for (int qi = 0; qi < 4; ++qi) {
            int rank = 0;
#pragma unroll
            for (int qj = 0; qj < 4; ++qj)
                rank += (qj != qi) && (len[qj] > len[qi] || (len[qj] == len[qi] && qj < qi));
            if (ok[qi]) { list |= qi << (2 * rank); ++nq; }
        }
        wbits = (U.w[0] > 1.5f ? 1 : 0) | (U.w[1] > 1.5f ? 2 : 0) | (V.w[0] > 1.5f ? 4 : 0) |
                (V.w[1] > 1.5f ? 8 : 0);
        box[0 * STRIDE] = U.lo[0]; box[1 * STRIDE] = U.hi[0];
        box[2 * STRIDE] = U.lo[1]; box[3 * STRIDE] = U.hi[1];
        box[4 * STRIDE] = V.lo[0]; box[5 * STRIDE] = V.hi[0];
        box[6 * STRIDE] = V.lo[1]; box[7 * STRIDE] = V.hi[1];
    }
    __device__ __forceinline__ void quadrant(int qi, double& a, double& b, double& c, double& d, double& w) const
    {
        const int i = qi >> 1, j = qi & 1;
        a = box[(2 * i) * STRIDE]; b = box[(2 * i + 1) * STRIDE];
        c = box[(4 + 2 * j) * STRIDE]; d = box[(5 + 2 * j) * STRIDE];
        w = (double)((1 + ((wbits >> i) & 1)) * (1 + ((wbits >> (2 + j)) & 1)));
    }
    // bins wlo .. whi of each quadrant reach the sink; each edge is evaluated
    // on its own, so the walk starts at max(mfirst, wlo)
    template <class Sink>
    __device__ __forceinline__ void sweep(int wlo, int whi, Sink& sink, double r0)
    {
#pragma unroll 1
        for (int t = 0; t < nq; ++t) {
            double a, b, c, d, w;
            quadrant((list >> (2 * t)) & 3, a, b, c, d, w);
            CyQuad q;
            cy_setup(q, P, a, b, c, d, r0);
            cy_sweep<NW, IL>(q, P, r0, wlo, whi, w, sink);
        }
    }
};

// Cylinder areas are FP64 in both variants.  With FP32 input and output one
// correction step after the FP32 seeds of the square roots and reciprocals
// (2^-46 after it) is enough; the FP64 variant takes two after the FP64 ones.
template <class Real> struct CylNewton { static constexpr int value = 2; };
template <> struct CylNewton<float> { static constexpr int value = 1; };

// IL: how the cylinder's I_l is evaluated (kIlExact, kIlTrapezoid, kIlTable);
// the planar I_l is exact either way
template <int SHAPE, class AT, class Real, int IL, int STRIDE = kThreads> struct PairOf;
template <class AT, class Real, int IL, int STRIDE> struct PairOf<0, AT, Real, IL, STRIDE> {
    using type = PlanarPair<AT>;
};
template <class AT, class Real, int IL, int STRIDE> struct PairOf<1, AT, Real, IL, STRIDE> {
    using type = CylinderPair<CylNewton<Real>::value, IL, STRIDE>;
};

// ---------------------------------------------------------------------------
// forward, closed-form areas
// ---------------------------------------------------------------------------

// sparse forward: transducers per work item, and the strided grid in units of
// 256 threads (4 x 4096 one-wave work-groups: 64 waves per CU at 256 CUs)
constexpr int kSparseChunk = 16;
constexpr int kSparseGrid = 4096;

// Waves per SIMD the closed-form kernels are built for (one-wave work-groups in
// the dense and sparse forward and the adjoint, 256-thread ones in the time
// tiles).  Cylinders for one or two volumes: four, in 128 VGPRs with a few
// spills outside the sweep; with more volumes the spills grow (120-210 bytes
// per lane) and they keep three.  The planar sweep in FP64 for four or eight
// volumes spills 300 bytes per lane at three and runs faster at two (1.75x for
// the adjoint of eight volumes); for one volume three is faster despite its
// spills (9 %).  The FP32 planar kernels fit four waves without spills
// (112-125 VGPRs).
template <int SHAPE, class AT, int NB>
constexpr int closed_waves()
{
    return SHAPE == 1 ? (NB <= 2 ? 4 : 3) : (sizeof(AT) == 8 ? (NB >= 4 ? 2 : 3) : (NB <= 2 ? 4 : 3));
}

// ---------------------------------------------------------------------------
// forward, closed-form areas, one wave per work-group
// ---------------------------------------------------------------------------

constexpr int kWave = 64;          // threads of a one-wave work-group: a 4 x 4 x 4 voxel cube

// LDS window of a one-wave work-group, in bytes, shared by its volumes: with
// sixteen of them per CU (four waves per SIMD) each may hold 10 KB; the
// cylinder kernels also keep their 4 KB table of interval ends there
template <int SHAPE>
constexpr int wave_window_bytes()
{
    return SHAPE == 1 ? 4096 : 8192;
}

// The wave's 64 voxels (one per lane; `valid` false for lanes without one)
// against transducers kperm[kbeg .. kend): per transducer the window is the
// union of the lanes' pair ranges, swept in passes of HW shells.  The wave owns
// its LDS window: it clears it, sweeps into it and adds it to f with no
// work-group barrier, only the ordering of its own LDS operations.
template <int SHAPE, class AT, int NB, class Real, int IL>
__device__ __forceinline__ void fwd_wave_voxels(const KParams& P, int ix, int iy, int iz, bool valid, int64_t idx,
                                                int kbeg, int kend, const Real* __restrict__ coef,
                                                double* __restrict__ f, double* hist, double* box)
{
    constexpr int HE = wave_window_bytes<SHAPE>() / (int)sizeof(double);
    constexpr int HW = HE / NB;          // shells per pass
    const int l = threadIdx.x;
    double p0[NB];
    bool nz = false;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        p0[b] = valid ? (double)coef[b * P.N + idx] : 0.0;
        nz |= p0[b] != 0.0;
    }
    if (!__any(nz)) return;
    const int S = P.step;
    const int64_t Mhi = P.Mlo + P.Mcount - 1;
    for (int kk = kbeg; kk < kend; ++kk) {
        const int k = P.kperm[kk];
        int wlo, whi;
        typename PairOf<SHAPE, AT, Real, IL, kWave>::type pair;
        pair.bind(box, P.lut);
        {
            const TrDev T = P.tr[k];
            double x[3];
            frame_coords(T, ix, iy, iz, x);
            int lo = 0x7fffffff, hi = -0x7fffffff - 1;
            if (nz) pair_range(T, x, P.r0, lo, hi);   // lanes whose volumes are all zero add nothing
            wave_window(P, lo, hi, wlo, whi);
            pair.setup(T, x, P.r0);
        }
        for (int plo = wlo; plo <= whi; plo += HW) {
            const int phi = min(whi, plo + HW - 1);
            const int wn = phi - plo + 1;
            for (int i = l; i < wn; i += kWave)
#pragma unroll
                for (int b = 0; b < NB; ++b) hist[b * HW + i] = 0.0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (nz) {
                auto sink = [&](int m, auto area) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) atomicAdd(&hist[b * HW + (m - plo)], p0[b] * (double)area);
                };
                pair.sweep(plo, phi, sink, P.r0);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i = l; i < wn * S; i += kWave) {
                const int jj = i / S;
                const int64_t m = (int64_t)(plo + jj - 1) * S + 1 + (i - jj * S);
                if (m < P.Mlo || m > Mhi) continue;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    double v = hist[b * HW + jj];
                    if (v != 0.0) unsafeAtomicAdd(&f[((int64_t)b * P.K + k) * P.Mcount + (m - P.Mlo)], v * S);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Dense forward: one work-group of one wave per (4 x 4 x 4 voxel cube, chunk
// of transducers).
template <int SHAPE, class AT, int NB, class Real, int IL>
__global__ __launch_bounds__(kWave, (closed_waves<SHAPE, AT, NB>())) void k_fwd_wave(KParams P,
                                                                                     const Real* __restrict__ coef,
                                                                                     double* __restrict__ f)
{
    __shared__ double hist[wave_window_bytes<SHAPE>() / sizeof(double)];   // [NB][shells per pass]
    __shared__ double box[SHAPE == 1 ? kBoxSlots * kWave : 1];
    const int ncx = (int)((P.n[0] + 3) / 4), ncy = (int)((P.n[1] + 3) / 4);
    const int cid = blockIdx.x;
    const int x0 = (cid % ncx) * 4, y0 = ((cid / ncx) % ncy) * 4, z0 = (cid / (ncx * ncy)) * 4;
    const int l = threadIdx.x;
    const int ix = x0 + (l & 3), iy = y0 + ((l >> 2) & 3), iz = z0 + (l >> 4);
    const bool valid = ix < P.n[0] && iy < P.n[1] && iz < P.n[2];
    const int64_t idx = valid ? ix + P.n[0] * (iy + P.n[1] * (int64_t)iz) : 0;
    const int kbeg = blockIdx.y * P.kchunk;
    fwd_wave_voxels<SHAPE, AT, NB, Real, IL>(P, ix, iy, iz, valid, idx, kbeg, min(P.nk, kbeg + P.kchunk), coef, f,
                                             hist, box);
}

// Sparse forward: work items (64 consecutive entries of the support list, a
// chunk of P.kchunk transducers), strided over a fixed grid of one-wave
// work-groups, since their number is known on the device only.  The list holds
// the nonzero voxels brick by brick in Morton order and, inside a brick, 4 x 4
// x 4 cube by cube, so 64 consecutive entries lie in a few neighbouring cubes
// and their pair ranges overlap.
template <int SHAPE, class AT, int NB, class Real, int IL>
__global__ __launch_bounds__(kWave, (closed_waves<SHAPE, AT, NB>())) void k_fwd_sparse_wave(
    KParams P, const Real* __restrict__ coef, double* __restrict__ f)
{
    __shared__ double hist[wave_window_bytes<SHAPE>() / sizeof(double)];   // [NB][shells per pass]
    __shared__ double box[SHAPE == 1 ? kBoxSlots * kWave : 1];
    const int64_t total = *P.sup_total;
    const int64_t nchunks = (P.nk + P.kchunk - 1) / P.kchunk;
    const int64_t items = (total + kWave - 1) / kWave * nchunks;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t g = it / nchunks;
        const int64_t e = g * kWave + threadIdx.x;
        const bool valid = e < total;
        const int64_t idx = valid ? (int64_t)P.sup_list[e] : 0;
        const int ix = (int)(idx % P.n[0]), iy = (int)((idx / P.n[0]) % P.n[1]), iz = (int)(idx / (P.n[0] * P.n[1]));
        const int kbeg = (int)(it % nchunks) * P.kchunk;
        fwd_wave_voxels<SHAPE, AT, NB, Real, IL>(P, ix, iy, iz, valid, idx, kbeg, min(P.nk, kbeg + P.kchunk), coef,
                                                 f, hist, box);
    }
}

// ---------------------------------------------------------------------------
// forward, closed-form areas, by (transducer, time tile): output-stationary
// ---------------------------------------------------------------------------

// One work-group per (transducer, tile of `tile` consecutive shells).  It owns
// the tile's fine bins of f for every volume of the launch, so f needs neither
// a fill nor atomics: the group scans the bricks, keeps those whose window
// meets the tile, and for each runs the pair setup and the sweep clipped to
// the tile into its LDS histogram, then stores the tile.  Work items come in
// the order of items[] (estimated cost, largest first) so that the in-order
// dispatch of work-groups balances the tail of the launch.
template <int SHAPE, class AT, int NB, class Real, int IL>
__global__ __launch_bounds__(kThreads, (closed_waves<SHAPE, AT, NB>())) void k_fwd_tile(
    KParams P, const int32_t* __restrict__ items, int tile, int ntiles, int nbricks, const Real* __restrict__ coef,
    double* __restrict__ f)
{
    extern __shared__ double hist[];   // [NB][tile]
    __shared__ double box[SHAPE == 1 ? kBoxSlots * kThreads : 1];
    __shared__ int cand[kThreads];
    __shared__ int ncand;
    const int item = items[blockIdx.x];
    const int kk = item / ntiles, t = item - kk * ntiles;
    const int k = P.kperm[kk];
    const int tlo = (int)P.Jlo + t * tile;
    const int thi = min((int)P.Jhi, tlo + tile - 1);
    for (int i = threadIdx.x; i < NB * tile; i += kThreads) hist[i] = 0.0;
    for (int c0 = 0; c0 < nbricks; c0 += kThreads) {
        const int b = c0 + threadIdx.x;
        bool hit = false;
        if (b < nbricks) {
            double lo[3], hi[3];
            brick_box(P, b, lo, hi);
            int wlo, whi;
            box_window(P, lo, hi, P.tr[k], wlo, whi);
            hit = wlo <= thi && whi >= tlo;
        }
        __syncthreads();   // the previous list has been consumed (the histogram cleared)
        if (threadIdx.x == 0) ncand = 0;
        __syncthreads();
        if (hit) cand[atomicAdd(&ncand, 1)] = b;
        __syncthreads();
        const int nc = ncand;
        for (int i = 0; i < nc; ++i) {
            Brick Bk;
            brick_setup(P, cand[i], Bk);
            double p0[NB];
            bool nz = false;
#pragma unroll
            for (int v = 0; v < NB; ++v) {
                p0[v] = Bk.valid ? (double)coef[v * P.N + Bk.idx] : 0.0;
                nz |= p0[v] != 0.0;
            }
            if (!__syncthreads_or(nz)) continue;
            typename PairOf<SHAPE, AT, Real, IL>::type pair;
            pair.bind(box, P.lut);
            {
                const TrDev T = P.tr[k];
                double x[3];
                frame_coords(T, Bk.ix, Bk.iy, Bk.iz, x);
                pair.setup(T, x, P.r0);
            }
            if (nz) {
                auto sink = [&](int m, auto area) {
#pragma unroll
                    for (int v = 0; v < NB; ++v) atomicAdd(&hist[v * tile + (m - tlo)], p0[v] * (double)area);
                };
                // planar quadrants are walked from their first bin whatever
                // the tile, and a cylinder walk evaluates each edge on its own
                // (the edges outside its quadrant set as in the cube forward):
                // the areas are the cube forward's bit for bit
                pair.sweep(tlo, thi, sink, P.r0);
            }
        }
    }
    __syncthreads();
    // shell j holds the fine bins (j - 1) step + 1 .. j step, its area split
    // evenly over them (Remark 1), as in the cube forward
    const int S = P.step;
    const int64_t Mhi = P.Mlo + P.Mcount - 1;
    const int wn = thi - tlo + 1;
    for (int i = threadIdx.x; i < wn * S; i += kThreads) {
        const int jj = i / S;
        const int64_t m = (int64_t)(tlo + jj - 1) * S + 1 + (i - jj * S);
        if (m < P.Mlo || m > Mhi) continue;
#pragma unroll
        for (int v = 0; v < NB; ++v) f[((int64_t)v * P.K + k) * P.Mcount + (m - P.Mlo)] = hist[v * tile + jj] * S;
    }
}

// Estimated work of each (transducer, time tile) item of a shape group: the
// shells of every brick's window that fall in the tile, summed over the bricks
// (integers, so the FP64 sums are exact and independent of their order).
// One thread per (brick, transducer); cost[kk ntiles + t].
__global__ __launch_bounds__(kThreads) void k_tile_cost(KParams P, int nbricks, int tile, int ntiles,
                                                        double* __restrict__ cost)
{
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= (int64_t)nbricks * P.nk) return;
    const int b = (int)(g % nbricks), kk = (int)(g / nbricks);
    double lo[3], hi[3];
    brick_box(P, b, lo, hi);
    int wlo, whi;
    box_window(P, lo, hi, P.tr[P.kperm[kk]], wlo, whi);
    if (wlo > whi) return;
    const int J0 = (int)P.Jlo;
    for (int t = (wlo - J0) / tile; t <= (whi - J0) / tile; ++t) {
        const int a = max(wlo, J0 + t * tile), z = min(whi, J0 + t * tile + tile - 1);
        atomicAdd(&cost[(int64_t)kk * ntiles + t], (double)(z - a + 1));
    }
}

// ---------------------------------------------------------------------------
// adjoint, closed-form areas
// ---------------------------------------------------------------------------

// One work-group of one wave per (4 x 4 x 4 voxel cube, chunk of transducers):
// the wave stages its own window of W in LDS and gathers, with no work-group
// barrier, only the ordering of its own LDS operations.
template <int SHAPE, class AT, int NB, class Real, int IL>
__global__ __launch_bounds__(kWave, (closed_waves<SHAPE, AT, NB>())) void k_adj_wave(KParams P,
                                                                                     const Real* __restrict__ W,
                                                                                     Real* __restrict__ out,
                                                                                     double* __restrict__ z64,
                                                                                     int direct)
{
    constexpr int HE = wave_window_bytes<SHAPE>() / (int)sizeof(Real);
    __shared__ Real Ws[HE];              // [NB][HB]
    constexpr int HB = HE / NB;          // shells per pass
    __shared__ double box[SHAPE == 1 ? kBoxSlots * kWave : 1];
    const int ncx = (int)((P.n[0] + 3) / 4), ncy = (int)((P.n[1] + 3) / 4);
    const int cid = blockIdx.x;
    const int x0 = (cid % ncx) * 4, y0 = ((cid / ncx) % ncy) * 4, z0 = (cid / (ncx * ncy)) * 4;
    const int l = threadIdx.x;
    const int ix = x0 + (l & 3), iy = y0 + ((l >> 2) & 3), iz = z0 + (l >> 4);
    const bool valid = ix < P.n[0] && iy < P.n[1] && iz < P.n[2];
    const int64_t idx = valid ? ix + P.n[0] * (iy + P.n[1] * (int64_t)iz) : 0;
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
    const int kbeg = blockIdx.y * P.kchunk, kend = min(P.nk, kbeg + P.kchunk);
    const int S = P.step;
    const int64_t Mhi = P.Mlo + P.Mcount - 1;
    for (int kk = kbeg; kk < kend; ++kk) {
        const int k = P.kperm[kk];
        int wlo, whi;
        typename PairOf<SHAPE, AT, Real, IL, kWave>::type pair;
        pair.bind(box, P.lut);
        {
            const TrDev T = P.tr[k];
            double x[3];
            frame_coords(T, ix, iy, iz, x);
            int lo = 0x7fffffff, hi = -0x7fffffff - 1;
            if (valid) pair_range(T, x, P.r0, lo, hi);
            wave_window(P, lo, hi, wlo, whi);
            pair.setup(T, x, P.r0);
        }
        for (int plo = wlo; plo <= whi; plo += HB) {
            const int phi = min(whi, plo + HB - 1);
            const int wn = phi - plo + 1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // transpose of the even split: each shell gathers its fine bins (Remark 1)
            for (int i = l; i < wn; i += kWave)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const Real* Wk = W + ((int64_t)b * P.K + k) * P.Mcount;
                    double a = 0.0;
                    for (int t = 0; t < S; ++t) {
                        const int64_t m = (int64_t)(plo + i - 1) * S + 1 + t;
                        if (m >= P.Mlo && m <= Mhi) a += (double)Wk[m - P.Mlo];
                    }
                    Ws[b * HB + i] = (Real)(a * S);
                }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid) {
                AT part[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) part[b] = AT(0);
                auto sink = [&](int m, auto area) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) part[b] = fma((AT)area, (AT)Ws[b * HB + (m - plo)], part[b]);
                };
                pair.sweep(plo, phi, sink, P.r0);
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[b] += (double)part[b];
            }
        }
    }
    if (!valid) return;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (direct) out[b * P.N + idx] = (Real)acc[b];
        else unsafeAtomicAdd(&z64[b * P.N + idx], acc[b]);
    }
}

// ---------------------------------------------------------------------------
// quadrature over surface points (Alg. 2 / Alg. 6)
// ---------------------------------------------------------------------------

// bin of the distance sqrt(r2): [r0 + m - 1, r0 + m); FP32 estimate, FP64
// decision.  The estimate is the one v_sqrt_f32 (1 ulp; the correctly rounded
// sqrtf the compiler would emit costs some 15 more instructions per point): at
// any distance here it lands within one bin of the true one, which the two FP64
// comparisons then correct
__device__ __forceinline__ int point_bin(double r2, double r0, float r0f)
{
    float rf = __builtin_amdgcn_sqrtf((float)r2);
    int m = (int)floorf(rf - r0f) + 1;
    double e = r0 + (double)(m - 1);
    if (r2 < e * e) return m - 1;
    e += 1.0;
    if (!(r2 < e * e)) return m + 1;
    return m;
}

template <class AT> __device__ __forceinline__ AT inv_dist(double r2);
template <> __device__ __forceinline__ float inv_dist<float>(double r2) { return __builtin_amdgcn_rsqf((float)r2); }
template <> __device__ __forceinline__ double inv_dist<double>(double r2) { return rsq64(r2); }

template <class AT, int NB, class Real>
__global__ __launch_bounds__(kThreads) void k_fwd_quad(KParams P, const Real* __restrict__ coef,
                                                        double* __restrict__ f)
{
    constexpr int HB = kHistQuad;   // bins per pass
    extern __shared__ double hist[];
    Brick Bk;
    brick_setup(P, blockIdx.x, Bk);
    double p0[NB];
    bool nz = false;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        p0[b] = Bk.valid ? (double)coef[b * P.N + Bk.idx] : 0.0;
        nz |= p0[b] != 0.0;
    }
    const double X0 = P.origin[0] + Bk.ix * P.w, X1 = P.origin[1] + Bk.iy * P.w, X2 = P.origin[2] + Bk.iz * P.w;
    if (!__syncthreads_or(nz)) return;
    const float r0f = (float)P.r0;
    const int kbeg = blockIdx.y * P.kchunk, kend = min(P.nk, kbeg + P.kchunk);
    for (int kk = kbeg; kk < kend; ++kk) {
        const int k = P.kperm[kk];
        const TrDev T = P.tr[k];
        const double* __restrict__ Q = P.qpts + (int64_t)k * P.Q * 3;
        const AT dA = (AT)P.qdA[k];
        int wlo, whi;
        brick_window(P, Bk, T, wlo, whi);
        for (int plo = wlo; plo <= whi; plo += HB) {
            const int phi = min(whi, plo + HB - 1);
            const int wn = phi - plo + 1;
            for (int i = threadIdx.x; i < wn; i += kThreads)
#pragma unroll
                for (int b = 0; b < NB; ++b) hist[b * HB + i] = 0.0;
            __syncthreads();
            if (nz) {
                int mcur = -(1 << 30);
                AT acc = AT(0);
                for (int q = 0; q < P.Q; ++q) {
                    double dx = Q[3 * q] - X0, dy = Q[3 * q + 1] - X1, dz = Q[3 * q + 2] - X2;
                    double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    int m = point_bin(r2, P.r0, r0f);
                    AT cv = dA * inv_dist<AT>(r2);
                    if (m != mcur) {
                        if (mcur >= plo && mcur <= phi)
#pragma unroll
                            for (int b = 0; b < NB; ++b) atomicAdd(&hist[b * HB + (mcur - plo)], p0[b] * (double)acc);
                        mcur = m;
                        acc = cv;
                    } else {
                        acc += cv;
                    }
                }
                if (mcur >= plo && mcur <= phi)
#pragma unroll
                    for (int b = 0; b < NB; ++b) atomicAdd(&hist[b * HB + (mcur - plo)], p0[b] * (double)acc);
            }
            __syncthreads();
            const int64_t fo = (plo - P.Mlo);
            for (int i = threadIdx.x; i < wn; i += kThreads)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    double v = hist[b * HB + i];
                    if (v != 0.0) unsafeAtomicAdd(&f[((int64_t)b * P.K + k) * P.Mcount + fo + i], v);
                }
            __syncthreads();
        }
    }
}

template <class AT, int NB, class Real>
__global__ __launch_bounds__(kThreads) void k_adj_quad(KParams P, const Real* __restrict__ W,
                                                        Real* __restrict__ out, double* __restrict__ z64,
                                                        int direct)
{
    constexpr int HB = kHistQuad;   // bins per pass
    extern __shared__ double smem_d[];
    Real* Ws = reinterpret_cast<Real*>(smem_d);
    Brick Bk;
    brick_setup(P, blockIdx.x, Bk);
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
    const double X0 = P.origin[0] + Bk.ix * P.w, X1 = P.origin[1] + Bk.iy * P.w, X2 = P.origin[2] + Bk.iz * P.w;
    const float r0f = (float)P.r0;
    const int kbeg = blockIdx.y * P.kchunk, kend = min(P.nk, kbeg + P.kchunk);
    for (int kk = kbeg; kk < kend; ++kk) {
        const int k = P.kperm[kk];
        const TrDev T = P.tr[k];
        const double* __restrict__ Q = P.qpts + (int64_t)k * P.Q * 3;
        const AT dA = (AT)P.qdA[k];
        int wlo, whi;
        brick_window(P, Bk, T, wlo, whi);
        for (int plo = wlo; plo <= whi; plo += HB) {
            const int phi = min(whi, plo + HB - 1);
            const int wn = phi - plo + 1;
            __syncthreads();
            const int64_t fo = (plo - P.Mlo);
            for (int i = threadIdx.x; i < wn; i += kThreads)
#pragma unroll
                for (int b = 0; b < NB; ++b) Ws[b * HB + i] = W[((int64_t)b * P.K + k) * P.Mcount + fo + i];
            __syncthreads();
            if (Bk.valid) {
                AT part[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) part[b] = AT(0);
                for (int q = 0; q < P.Q; ++q) {
                    double dx = Q[3 * q] - X0, dy = Q[3 * q + 1] - X1, dz = Q[3 * q + 2] - X2;
                    double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    int m = point_bin(r2, P.r0, r0f);
                    if (m < plo || m > phi) continue;
                    AT cv = dA * inv_dist<AT>(r2);
#pragma unroll
                    for (int b = 0; b < NB; ++b) part[b] = fma(cv, (AT)Ws[b * HB + (m - plo)], part[b]);
                }
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[b] += (double)part[b];
            }
        }
    }
    if (!Bk.valid) return;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (direct) out[b * P.N + Bk.idx] = (Real)acc[b];
        else unsafeAtomicAdd(&z64[b * P.N + Bk.idx], acc[b]);
    }
}

// ---------------------------------------------------------------------------
// work count: area evaluations (closed form: one per quadrant and bin inside the
// kept range; quadrature: one per surface point) and voxel-transducer pairs
// ---------------------------------------------------------------------------

template <int SHAPE>
__global__ __launch_bounds__(kThreads) void k_count(KParams P, int quad, unsigned long long* __restrict__ out)
{
    __shared__ unsigned long long red[2];
    __shared__ double box[SHAPE == 1 ? kBoxSlots * kThreads : 1];
    if (threadIdx.x < 2) red[threadIdx.x] = 0;
    __syncthreads();
    Brick Bk;
    brick_setup(P, blockIdx.x, Bk);
    unsigned long long evals = 0, pairs = 0;
    if (Bk.valid) {
        for (int kk = 0; kk < P.nk; ++kk) {
            const TrDev T = P.tr[P.kperm[kk]];
            if (quad) { evals += P.Q; pairs += 1; continue; }
            double x[3];
            frame_coords(T, Bk.ix, Bk.iy, Bk.iz, x);
            const int lo = (int)P.Jlo, hi = (int)P.Jhi;
            int nb = 0;
            auto sink = [&](int, auto) { ++nb; };
            typename PairOf<SHAPE, double, double, kIlExact>::type pair;
            pair.bind(box, nullptr);
            pair.setup(T, x, P.r0);
            pair.sweep(lo, hi, sink, P.r0);
            evals += nb;
            pairs += 1;
        }
    }
    atomicAdd(&red[0], evals);
    atomicAdd(&red[1], pairs);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], red[0]);
        atomicAdd(&out[1], red[1]);
    }
}

// ---------------------------------------------------------------------------
// support of the coefficients (the voxels the forward's sum over voxels needs)
// ---------------------------------------------------------------------------

template <class Real>
__device__ __forceinline__ bool voxel_nonzero(const KParams& P, const Brick& Bk, const Real* coef, int B)
{
    bool nz = false;
    if (Bk.valid)
        for (int b = 0; b < B; ++b) nz |= coef[b * P.N + Bk.idx] != Real(0);
    return nz;
}

// nonzero voxels per brick
template <class Real>
__global__ __launch_bounds__(kThreads) void k_support_count(KParams P, const Real* __restrict__ coef, int B,
                                                             const int32_t* __restrict__ order,
                                                             int32_t* __restrict__ cnt)
{
    Brick Bk;
    brick_setup(P, order[blockIdx.x], Bk);
    const int c = __syncthreads_count(voxel_nonzero(P, Bk, coef, B));
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

// exclusive prefix sums of the per-brick counts (one work-group); off[n] = total
__global__ __launch_bounds__(kThreads) void k_support_scan(const int32_t* __restrict__ cnt, int n,
                                                            int32_t* __restrict__ off)
{
    __shared__ int s[kThreads];
    int carry = 0;
    for (int base = 0; base < n; base += kThreads) {
        const int i = base + threadIdx.x;
        const int v = i < n ? cnt[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kThreads; o <<= 1) {
            const int t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) off[i] = carry + s[threadIdx.x] - v;
        carry += s[kThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[n] = carry;
}

// the nonzero voxels of each brick at the brick's offset, in thread order (the
// brick's four 4 x 4 x 4 cubes in turn); bricks in the order `order` (Morton
// order of the brick coordinates, so that consecutive entries lie in a compact
// cluster of bricks)
template <class Real>
__global__ __launch_bounds__(kThreads) void k_support_write(KParams P, const Real* __restrict__ coef, int B,
                                                             const int32_t* __restrict__ order,
                                                             const int32_t* __restrict__ off,
                                                             int32_t* __restrict__ list)
{
    __shared__ int wcount[kThreads / 64];
    Brick Bk;
    brick_setup(P, order[blockIdx.x], Bk);
    const bool nz = voxel_nonzero(P, Bk, coef, B);
    const unsigned long long m = __ballot(nz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[w] = __popcll(m);
    __syncthreads();
    int base = off[blockIdx.x];
    for (int v = 0; v < w; ++v) base += wcount[v];
    if (nz) list[base + rank] = (int32_t)Bk.idx;
}

// ---------------------------------------------------------------------------
// temporal stage
// ---------------------------------------------------------------------------

// s_hat[b][k][l] = sum_j G[j] scale[m] f[b][k][m],  m = U l - (jlo + jj)  (0-based l)
template <class Real>
__global__ void k_fir(const double* __restrict__ f, const double* __restrict__ scale, const double* __restrict__ G,
                      int jlo, int jcnt, int U, int L, int K, int64_t Mlo, int64_t Mcount, Real* __restrict__ out)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y, b = blockIdx.z;
    if (l >= L) return;
    const double* fk = f + ((int64_t)b * K + k) * Mcount;
    // h sums to zero, so the samples are small differences of large terms:
    // accumulated in FP64
    double acc = 0.0;
    const int64_t mtop = (int64_t)U * l - jlo;   // m for jj = 0
    for (int jj = 0; jj < jcnt; ++jj) {
        int64_t mi = mtop - jj - Mlo;
        if (mi < 0 || mi >= Mcount) continue;
        acc = fma(G[jj], scale[mi] * fk[mi], acc);
    }
    out[((int64_t)b * K + k) * L + l] = (Real)acc;
}

// W[b][k][m] = scale[m] sum_l G[U l - m] y[b][k][l]
template <class Real>
__global__ void k_adjw(const Real* __restrict__ y, const double* __restrict__ scale, const double* __restrict__ G,
                       int jlo, int jcnt, int U, int L, int K, int64_t Mlo, int64_t Mcount, Real* __restrict__ W)
{
    const int64_t mi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int k = blockIdx.y, b = blockIdx.z;
    if (mi >= Mcount) return;
    const int m = (int)(Mlo + mi);
    const Real* yk = y + ((int64_t)b * K + k) * L;
    // U l - m = j in [jlo, jlo + jcnt - 1]
    int lmin = -floordiv(-(m + jlo), U);
    int lmax = floordiv(m + jlo + jcnt - 1, U);
    lmin = max(lmin, 0);
    lmax = min(lmax, L - 1);
    double acc = 0.0;
    for (int l = lmin; l <= lmax; ++l) acc = fma(G[U * l - m - jlo], (double)yk[l], acc);
    W[((int64_t)b * K + k) * Mcount + mi] = (Real)(scale[mi] * acc);
}

// ---------------------------------------------------------------------------
// E~ / F~ tables of the lookup-table I_l, one node per thread
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_lut_build(double2* __restrict__ T)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= kLutN * kLutN) return;
    const double s = lut_node(id % kLutN), nu = lut_node(id / kLutN);
    double E = 0.0, F = 0.0;
    if (s > 0.0) {
        const double c = sqrt64<2>((1.0 - s) * (1.0 + s));   // cos(arcsin s)
        const double dl = sqrt64<2>(fma(-nu * s, s, 1.0));    // Delta(arcsin s)
        E = ellip_e_scd<2, true>(s, c, dl, nu, &F);
    }
    T[id] = make_double2(E, F);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

namespace {

template <int SHAPE, class AT, class Real, int IL>
hipError_t fwd_sparse_nb(int nb, dim3 grid, const KParams& P, const Real* coef, double* f, hipStream_t s)
{
    switch (nb) {
    case 1: k_fwd_sparse_wave<SHAPE, AT, 1, Real, IL><<<grid, kWave, 0, s>>>(P, coef, f); break;
    case 2: k_fwd_sparse_wave<SHAPE, AT, 2, Real, IL><<<grid, kWave, 0, s>>>(P, coef, f); break;
    case 4: k_fwd_sparse_wave<SHAPE, AT, 4, Real, IL><<<grid, kWave, 0, s>>>(P, coef, f); break;
    default: k_fwd_sparse_wave<SHAPE, AT, 8, Real, IL><<<grid, kWave, 0, s>>>(P, coef, f); break;
    }
    return hipGetLastError();
}

template <int SHAPE, class AT, class Real, int IL>
hipError_t fwd_wave_nb(int nb, dim3 grid, const KParams& P, const Real* coef, double* f, hipStream_t s)
{
    switch (nb) {
    case 1: k_fwd_wave<SHAPE, AT, 1, Real, IL><<<grid, kWave, 0, s>>>(P, coef, f); break;
    case 2: k_fwd_wave<SHAPE, AT, 2, Real, IL><<<grid, kWave, 0, s>>>(P, coef, f); break;
    case 4: k_fwd_wave<SHAPE, AT, 4, Real, IL><<<grid, kWave, 0, s>>>(P, coef, f); break;
    default: k_fwd_wave<SHAPE, AT, 8, Real, IL><<<grid, kWave, 0, s>>>(P, coef, f); break;
    }
    return hipGetLastError();
}

template <int SHAPE, class AT, class Real, int IL>
hipError_t adj_wave_nb(int nb, dim3 grid, const KParams& P, const Real* W, Real* out, double* z64, int direct,
                       hipStream_t s)
{
    switch (nb) {
    case 1: k_adj_wave<SHAPE, AT, 1, Real, IL><<<grid, kWave, 0, s>>>(P, W, out, z64, direct); break;
    case 2: k_adj_wave<SHAPE, AT, 2, Real, IL><<<grid, kWave, 0, s>>>(P, W, out, z64, direct); break;
    case 4: k_adj_wave<SHAPE, AT, 4, Real, IL><<<grid, kWave, 0, s>>>(P, W, out, z64, direct); break;
    default: k_adj_wave<SHAPE, AT, 8, Real, IL><<<grid, kWave, 0, s>>>(P, W, out, z64, direct); break;
    }
    return hipGetLastError();
}

template <int SHAPE, class AT, class Real, int IL>
hipError_t fwd_tile_nb(int nb, const KParams& P, const int32_t* items, int nitems, int tile, int ntiles,
                       int nbricks, const Real* coef, double* f, hipStream_t s)
{
    const size_t sh = (size_t)nb * tile * sizeof(double);
    switch (nb) {
    case 1: k_fwd_tile<SHAPE, AT, 1, Real, IL><<<nitems, kThreads, sh, s>>>(P, items, tile, ntiles, nbricks, coef, f); break;
    case 2: k_fwd_tile<SHAPE, AT, 2, Real, IL><<<nitems, kThreads, sh, s>>>(P, items, tile, ntiles, nbricks, coef, f); break;
    case 4: k_fwd_tile<SHAPE, AT, 4, Real, IL><<<nitems, kThreads, sh, s>>>(P, items, tile, ntiles, nbricks, coef, f); break;
    default: k_fwd_tile<SHAPE, AT, 8, Real, IL><<<nitems, kThreads, sh, s>>>(P, items, tile, ntiles, nbricks, coef, f); break;
    }
    return hipGetLastError();
}

template <class Real>
hipError_t fwd_tile_cyl(int mode, int nb, const KParams& P, const int32_t* items, int nitems, int tile, int ntiles,
                        int nbricks, const Real* coef, double* f, hipStream_t s)
{
    if (mode == 2)
        return fwd_tile_nb<1, double, Real, kIlTrapezoid>(nb, P, items, nitems, tile, ntiles, nbricks, coef, f, s);
    if (mode == 3)
        return fwd_tile_nb<1, double, Real, kIlTable>(nb, P, items, nitems, tile, ntiles, nbricks, coef, f, s);
    return fwd_tile_nb<1, double, Real, kIlExact>(nb, P, items, nitems, tile, ntiles, nbricks, coef, f, s);
}

// cylinder launches by I_l variant: area mode 0 exact, 2 trapezoid, 3 tables
template <class Real>
hipError_t fwd_sparse_cyl(int mode, int nb, dim3 grid, const KParams& P, const Real* coef, double* f, hipStream_t s)
{
    if (mode == 2) return fwd_sparse_nb<1, double, Real, kIlTrapezoid>(nb, grid, P, coef, f, s);
    if (mode == 3) return fwd_sparse_nb<1, double, Real, kIlTable>(nb, grid, P, coef, f, s);
    return fwd_sparse_nb<1, double, Real, kIlExact>(nb, grid, P, coef, f, s);
}

template <class AT, class Real>
hipError_t fwd_quad_nb(int nb, dim3 grid, const KParams& P, const Real* coef, double* f, hipStream_t s)
{
    size_t sh = (size_t)nb * kHistQuad * sizeof(double);
    switch (nb) {
    case 1: k_fwd_quad<AT, 1, Real><<<grid, kThreads, sh, s>>>(P, coef, f); break;
    case 2: k_fwd_quad<AT, 2, Real><<<grid, kThreads, sh, s>>>(P, coef, f); break;
    case 4: k_fwd_quad<AT, 4, Real><<<grid, kThreads, sh, s>>>(P, coef, f); break;
    default: k_fwd_quad<AT, 8, Real><<<grid, kThreads, sh, s>>>(P, coef, f); break;
    }
    return hipGetLastError();
}

template <class AT, class Real>
hipError_t adj_quad_nb(int nb, dim3 grid, const KParams& P, const Real* W, Real* out, double* z64, int direct,
                       hipStream_t s)
{
    size_t sh = (size_t)nb * kHistQuad * sizeof(Real);
    switch (nb) {
    case 1: k_adj_quad<AT, 1, Real><<<grid, kThreads, sh, s>>>(P, W, out, z64, direct); break;
    case 2: k_adj_quad<AT, 2, Real><<<grid, kThreads, sh, s>>>(P, W, out, z64, direct); break;
    case 4: k_adj_quad<AT, 4, Real><<<grid, kThreads, sh, s>>>(P, W, out, z64, direct); break;
    default: k_adj_quad<AT, 8, Real><<<grid, kThreads, sh, s>>>(P, W, out, z64, direct); break;
    }
    return hipGetLastError();
}

int chunk_nb(int rem)
{
    return rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
}

int grid_fill_blocks(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

template <class Real>
hipError_t forward_t(const LaunchPlan& L, const Real* coef, Real* sig, int B, hipStream_t s, bool sparse)
{
    hipError_t e;
    // the (transducer, time tile) forward stores every fine bin of f itself
    const bool tiles = L.tile > 0 && !sparse && L.mode != 1;
    if (!tiles) {
        const int64_t nf = (int64_t)B * L.base.K * L.base.Mcount;
        k_fill<<<grid_fill_blocks(nf), 256, 0, s>>>(L.f, nf);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (sparse) {
        // support of the whole batch: the voxels with a nonzero coefficient in any volume
        k_support_count<Real><<<L.nbricks, kThreads, 0, s>>>(L.base, coef, B, L.sup_order, L.sup_cnt);
        k_support_scan<<<1, kThreads, 0, s>>>(L.sup_cnt, L.nbricks, L.sup_off);
        k_support_write<Real><<<L.nbricks, kThreads, 0, s>>>(L.base, coef, B, L.sup_order, L.sup_off, L.sup_list);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int b0 = 0; b0 < B;) {
        const int nb = chunk_nb(B - b0);
        for (int g = 0; g < L.ngroups; ++g) {
            const ShapeGroup& G = L.groups[g];
            KParams P = L.base;
            P.kperm = G.kperm;
            P.nk = G.nk;
            P.kchunk = G.kchunk_fwd;
            P.B = nb;
            dim3 grid(L.nbricks, (G.nk + G.kchunk_fwd - 1) / G.kchunk_fwd);
            const Real* cb = coef + (int64_t)b0 * P.N;
            double* fb = L.f + (int64_t)b0 * P.K * P.Mcount;
            if (sparse) {
                P.sup_list = L.sup_list;
                P.sup_total = L.sup_off + L.nbricks;
                P.kchunk = kSparseChunk;
                grid = dim3(kSparseGrid * (kThreads / kWave), 1);
            }
            if (L.mode == 1) e = fwd_quad_nb<Real, Real>(nb, grid, P, cb, fb, s);
            else if (tiles && G.shape == 0)
                e = fwd_tile_nb<0, Real, Real, kIlExact>(nb, P, G.items, G.nitems, L.tile, L.ntiles, L.nbricks, cb,
                                                         fb, s);
            else if (tiles)
                e = fwd_tile_cyl<Real>(L.mode, nb, P, G.items, G.nitems, L.tile, L.ntiles, L.nbricks, cb, fb, s);
            else if (sparse && G.shape == 0) e = fwd_sparse_nb<0, Real, Real, kIlExact>(nb, grid, P, cb, fb, s);
            else if (sparse) e = fwd_sparse_cyl<Real>(L.mode, nb, grid, P, cb, fb, s);
            else {
                const dim3 gw((unsigned)L.ncubes, (G.nk + G.kchunk_fwd - 1) / G.kchunk_fwd);
                if (G.shape == 0) e = fwd_wave_nb<0, Real, Real, kIlExact>(nb, gw, P, cb, fb, s);
                else if (L.mode == 2) e = fwd_wave_nb<1, double, Real, kIlTrapezoid>(nb, gw, P, cb, fb, s);
                else if (L.mode == 3) e = fwd_wave_nb<1, double, Real, kIlTable>(nb, gw, P, cb, fb, s);
                else e = fwd_wave_nb<1, double, Real, kIlExact>(nb, gw, P, cb, fb, s);
            }
            if (e != hipSuccess) return e;
        }
        b0 += nb;
    }
    dim3 g2((L.L + 255) / 256, L.base.K, B);
    k_fir<Real><<<g2, 256, 0, s>>>(L.f, L.scale, L.G, L.jlo, L.jcnt, L.U, L.L, L.base.K,
                                   L.base.Mlo, L.base.Mcount, sig);
    return hipGetLastError();
}

template <class Real>
hipError_t adjoint_t(const LaunchPlan& L, const Real* sig, Real* coef, int B, hipStream_t s)
{
    hipError_t e;
    Real* W = (Real*)L.W;
    dim3 g1((unsigned)((L.base.Mcount + 255) / 256), L.base.K, B);
    k_adjw<Real><<<g1, 256, 0, s>>>(sig, L.scale, L.G, L.jlo, L.jcnt, L.U, L.L, L.base.K,
                                    L.base.Mlo, L.base.Mcount, W);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    bool direct = L.ngroups == 1 && L.groups[0].kchunk_adj >= L.groups[0].nk;
    const int64_t nz = (int64_t)B * L.base.N;
    if (!direct) {
        k_fill<<<grid_fill_blocks(nz), 256, 0, s>>>(L.z64, nz);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (int b0 = 0; b0 < B;) {
        const int nb = chunk_nb(B - b0);
        for (int g = 0; g < L.ngroups; ++g) {
            const ShapeGroup& G = L.groups[g];
            KParams P = L.base;
            P.kperm = G.kperm;
            P.nk = G.nk;
            P.kchunk = G.kchunk_adj;
            P.B = nb;
            dim3 grid(L.nbricks, (G.nk + G.kchunk_adj - 1) / G.kchunk_adj);
            const Real* Wb = W + (int64_t)b0 * P.K * P.Mcount;
            Real* ob = coef + (int64_t)b0 * P.N;
            double* zb = L.z64 + (int64_t)b0 * P.N;
            if (L.mode == 1) e = adj_quad_nb<Real, Real>(nb, grid, P, Wb, ob, zb, direct, s);
            else {
                const dim3 gw((unsigned)L.ncubes, (G.nk + G.kchunk_adj - 1) / G.kchunk_adj);
                if (G.shape == 0) e = adj_wave_nb<0, Real, Real, kIlExact>(nb, gw, P, Wb, ob, zb, direct, s);
                else if (L.mode == 2) e = adj_wave_nb<1, double, Real, kIlTrapezoid>(nb, gw, P, Wb, ob, zb, direct, s);
                else if (L.mode == 3) e = adj_wave_nb<1, double, Real, kIlTable>(nb, gw, P, Wb, ob, zb, direct, s);
                else e = adj_wave_nb<1, double, Real, kIlExact>(nb, gw, P, Wb, ob, zb, direct, s);
            }
            if (e != hipSuccess) return e;
        }
        b0 += nb;
    }
    if (!direct) {
        k_finish<Real><<<grid_fill_blocks(nz), 256, 0, s>>>(L.z64, coef, nz);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_count(const LaunchPlan& L, unsigned long long* out, hipStream_t s)
{
    for (int g = 0; g < L.ngroups; ++g) {
        KParams P = L.base;
        P.kperm = L.groups[g].kperm;
        P.nk = L.groups[g].nk;
        if (L.groups[g].shape == 0) k_count<0><<<L.nbricks, kThreads, 0, s>>>(P, L.mode == 1, out);
        else k_count<1><<<L.nbricks, kThreads, 0, s>>>(P, L.mode == 1, out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tile_cost(const KParams& P, int nbricks, int tile, int ntiles, double* cost, hipStream_t s)
{
    const int64_t n = (int64_t)nbricks * P.nk;
    k_tile_cost<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(P, nbricks, tile, ntiles, cost);
    return hipGetLastError();
}

hipError_t launch_forward(const LaunchPlan& L, const void* coef, void* sig, int B, hipStream_t s)
{
    if (L.fp64) return forward_t<double>(L, (const double*)coef, (double*)sig, B, s, false);
    return forward_t<float>(L, (const float*)coef, (float*)sig, B, s, false);
}

hipError_t launch_lut_build(double2* table, hipStream_t s)
{
    k_lut_build<<<(kLutN * kLutN + 255) / 256, 256, 0, s>>>(table);
    return hipGetLastError();
}

hipError_t launch_forward_sparse(const LaunchPlan& L, const void* coef, void* sig, int B, hipStream_t s)
{
    if (L.mode == 1) return hipErrorNotSupported;
    if (L.fp64) return forward_t<double>(L, (const double*)coef, (double*)sig, B, s, true);
    return forward_t<float>(L, (const float*)coef, (float*)sig, B, s, true);
}

hipError_t launch_adjoint(const LaunchPlan& L, const void* sig, void* coef, int B, hipStream_t s)
{
    if (L.fp64) return adjoint_t<double>(L, (const double*)sig, (double*)coef, B, s);
    return adjoint_t<float>(L, (const float*)sig, (float*)coef, B, s);
}

}  // namespace patop
