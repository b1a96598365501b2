// Shell areas |M_i^m| of one voxel on one transducer, device side.
//
// A bin m is the radial interval [r0 + m - 1, r0 + m) in units of dr = c/(U fs).
// Both geometries use the paper's separable form (Sec. 4, Eq. separable): the
// squared distance is psi(u) + v^2 on a parameter rectangle D, which is split
// into at most four quadrants reflected to u, v >= 0 (Eq. uvminmax, folded
// intervals Eq. folded_intervals for the cylinder), each of the form
// [a, b] x [c, d].  A sweep walks the bins a quadrant touches (between its
// nearest corner distance D_ac and farthest D_bd, Eq. closedform_rminrmax) and
// hands each bin's area to a sink.
//
// Planar (Sec. 4.1): psi(u) = u^2 + x3^2, so in the plane of the rectangle the
// shell is the annulus s0 <= u^2 + v^2 < s1 with s = r^2 - x3^2.  The area of
// Eq. area_D_l_xi is evaluated in an equivalent form free of cancellation:
//   2 |D^m| = int_{s0}^{s1} Theta(s) ds,
// Theta(s) the angle subtended by the arc of radius sqrt(s) inside the
// quadrant.  Theta = theta_hi - theta_lo, where theta_hi is acos(a/sqrt s) up to
// the corner s_ad = a^2 + d^2 and asin(d/sqrt s) after it, theta_lo is
// asin(c/sqrt s) up to s_bc and acos(b/sqrt s) after it.  Between these
// breakpoints each term has the elementary antiderivative of Eq.
// plane_primitive, rearranged as
//   int_{s0}^{s1} acos(p/sqrt s) ds = (s1 - s0) acos(p/sqrt s1) + C,
//   int_{s0}^{s1} asin(p/sqrt s) ds = (s1 - s0) asin(p/sqrt s1) - C,
//   C = s0 (atan x - x) - x w0 dw,   w = sqrt(s - p^2), dw = w1 - w0,
//   x = p dw / (p^2 + w0 w1)      (tan of the angle swept between s0 and s1),
// so 2|D^m| = (s1 - s0) Theta(s1) + (corrections C), with Theta(s1) from one
// atan2 of the chord between the two arc end points and every difference of
// nearby squares taken from per-pair offsets that are exact to rounding.
//
// Cylinder (Sec. 4.2): psi(u) = (R - rho)^2 + 4 R rho sin^2(u/2).  Alg. 4 is
// followed literally (triples carried from edge to edge, Eq. area_D_l_xi,
// Eq. cyl_Il), in FP64: the cylinder's I_l is a difference of nearly equal
// elliptic integrals.  E(beta/2, nu) - E(alpha/2, nu) is evaluated by Legendre's
// addition theorem, E(phi) - E(psi) = E(sigma) - nu sin phi sin psi sin sigma, so
// only one Carlson evaluation, at the amplitude sigma of the difference, is needed
// (E = s R_F(c^2, 1 - nu s^2, 1) - nu/3 s^3 R_D(c^2, 1 - nu s^2, 1), valid for
// nu > 1 whenever nu s^2 <= 1, Lemma exact_integral).  The half angles of the
// clamped inverse Phi (Eq. alphabeta) come from
//   sin^2(u/2) = (s - v^2 - (R - rho)^2) / (4 R rho),
//   1 - nu sin^2(u/2) = v^2 / (s - (R - rho)^2),
// so arccos is never evaluated.
//
// Two cheaper I_l replace the Carlson evaluation (selected by IL): the chord of
// the level curve (Eq. trapezoid_Il) and the lookup tables of E~, F~ (Sec. 4.2,
// LUT paragraph), E(beta/2) - E(alpha/2) read off bilinearly at both end points.
#pragma once

#include <hip/hip_runtime.h>

#include "patop_internal.h"

namespace patop {

// ---------------------------------------------------------------------------
// small numeric helpers
// ---------------------------------------------------------------------------

// Seeds of the FP64 reciprocal and reciprocal square root.  NW = 1 (one
// correction step, the FP32-I/O cylinder kernels): the FP32 instructions
// v_rcp_f32 / v_rsq_f32 (1 ulp, 2^-23), which on gfx950 cost, with their two
// conversions, about half of v_rcp_f64 / v_rsq_f64; one Newton step then leaves
// 2^-46 (rcp) and 1.5 x 2^-46 (rsq) relative error.  Their arguments must lie
// in the FP32 normal range (or be <= 0 where the result is not used).  NW >= 2:
// the FP64 instructions (~2^-24), two steps to full precision.
template <int NW>
__device__ __forceinline__ double rcp_seed(double x)
{
    if (NW == 1) return (double)__builtin_amdgcn_rcpf((float)x);
    return __builtin_amdgcn_rcp(x);
}
template <int NW>
__device__ __forceinline__ double rsq_seed(double x)
{
    if (NW == 1) return (double)__builtin_amdgcn_rsqf((float)x);
    return __builtin_amdgcn_rsq(x);
}

// the offset that keeps square-root arguments positive (and, for NW = 1, in
// the FP32 normal range of the seeds); below any length or cosine that enters
// a sum here
template <int NW> struct Tiny { static constexpr double value = 1e-300; };
template <> struct Tiny<1> { static constexpr double value = 1e-30; };

// 1/x with one Newton step
template <int NW = 2>
__device__ __forceinline__ double rcp64(double x)
{
    double r = rcp_seed<NW>(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// a * b + c as one three-operand v_fma_f64 with the addend c in a register.
// Horner steps add a loop-invariant constant; left to itself the compiler
// copies it into the destination of a two-operand v_fmac_f64, one extra
// instruction per step.  b is a register too ("v") or, for a constant
// multiplier, a scalar register ("s").
__device__ __forceinline__ double fma_vvv(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ double fma_vsv(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// 1/x with a second Newton step (full precision)
__device__ __forceinline__ double rcp64_full(double x)
{
    double r = rcp64(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// v_rsq_f64 is accurate to ~2^-24: each Newton step doubles the correct bits
// (one step: ~2^-48, two: full precision)
template <int NEWTON = 2>
__device__ __forceinline__ double rsq64(double x)
{
    double r = rsq_seed<NEWTON>(x);
#pragma unroll
    for (int i = 0; i < NEWTON; ++i) {
        double h = 0.5 * x * r;
        r = fma(r, fma(-h, r, 0.5), r);
    }
    return r;
}

// sqrt of x > 0 from y = v_rsq_f64(x) (relative error ~2^-24): g = x y is
// corrected by the residual x - g^2 times h = y/2 (one step: ~2^-48); two
// steps first refine g and h together (Goldschmidt), then take the residual
// step (full precision)
template <int NEWTON = 2>
__device__ __forceinline__ double sqrt64_pos(double x)
{
    const double y = rsq_seed<NEWTON>(x);
    double g = x * y, h = 0.5 * y;
    if (NEWTON >= 2) {
        const double r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
    }
    return fma(fma(-g, g, x), h, g);
}

// sqrt(max(x, tiny)): branch free; returns sqrt(tiny) (1e-150, or 1e-15 with the
// FP32 seeds) instead of 0 for x <= 0, below any length or cosine that enters a
// sum here
template <int NEWTON = 2>
__device__ __forceinline__ double sqrt64(double x)
{
    return sqrt64_pos<NEWTON>(fmax(x, Tiny<NEWTON>::value));
}

// FP32 square root as the one v_sqrt_f32 (1 ulp); the IEEE-rounded sqrtf the
// compiler emits otherwise adds a denormal rescale and a correction step
// (some 15 instructions)
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(fmaxf(x, 0.0f)); }
__device__ __forceinline__ double sqrt_t(double x) { return x > 0.0 ? x * rsq64(x) : 0.0; }
// atan2 for y, x >= 0.  Small angles (y <= x/5) take the odd Taylor series of
// atan(y/x), whose error is the rounding of a few correctly rounded operations;
// the library routine's error, a smooth function of its argument, would be
// shared by neighbouring voxels and survive their summation into one bin.
__device__ __forceinline__ float atan2_t(float y, float x)
{
    if (y <= 0.2f * x) {
        float t = y * __builtin_amdgcn_rcpf(x), u = t * t;
        float p = fmaf(u, fmaf(u, fmaf(u, fmaf(u, fmaf(u, fmaf(u, 1.0f / 13, -1.0f / 11), 1.0f / 9), -1.0f / 7),
                                       1.0f / 5), -1.0f / 3), 1.0f);
        return t * p;
    }
    return atan2f(y, x);
}
__device__ __forceinline__ double atan2_t(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float atan_t(float x) { return atanf(x); }
__device__ __forceinline__ double atan_t(double x) { return atan(x); }

// 1/x from the hardware reciprocal: v_rcp_f32 (1 ulp) in FP32, v_rcp_f64 with
// two Newton steps in FP64
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// atan(x) - x and atan(x) for x >= 0, the first without cancellation: halving
//   atan x - x = 2 (atan y - y) - x^3 / (1 + sqrt(1 + x^2))^2,  y = x / (1 + sqrt(1 + x^2)),
// (atan x = 2 atan y) then the Taylor series of atan y - y, through y^13; its
// relative truncation error is ~0.2 y^12: below 1.2e-8 (FP32) from y < 0.25,
// below 2e-13 (the FP64 series runs to y^23) from y < 0.1.  Above 4 the
// library's atan gives both (there the difference has no cancellation).
template <class T>
struct AtanPair {
    T mx;   // atan x - x
    T a;    // atan x
};

template <class T> struct AtanMx;

template <> struct AtanMx<float> {
    static constexpr float kSmall = 0.25f;   // eval halves the angle from here on
    // x < kSmall: the series alone, which is what eval computes there
    static __device__ __forceinline__ AtanPair<float> small(float x)
    {
        float y = x * x;
        float p = fmaf(y, fmaf(y, fmaf(y, fmaf(y, fmaf(y, -1.0f / 13, 1.0f / 11), -1.0f / 9), 1.0f / 7), -1.0f / 5),
                       1.0f / 3);
        const float t = -x * y * p;
        return {t, x + t};
    }
    static __device__ __forceinline__ AtanPair<float> eval(float x)
    {
        if (x > 4.0f) {
            const float a = atanf(x);
            return {a - x, a};
        }
        const float x0 = x;
        float acc = 0.0f, scale = 1.0f;
        for (int i = 0; i < 4 && x >= 0.25f; ++i) {
            float q = 1.0f + __builtin_amdgcn_sqrtf(fmaf(x, x, 1.0f));
            float iq = __builtin_amdgcn_rcpf(q);
            acc = fmaf(-scale * x * x * x, iq * iq, acc);
            x *= iq;
            scale *= 2.0f;
        }
        float y = x * x;
        float p = fmaf(y, fmaf(y, fmaf(y, fmaf(y, fmaf(y, -1.0f / 13, 1.0f / 11), -1.0f / 9), 1.0f / 7), -1.0f / 5),
                       1.0f / 3);
        const float t = -scale * x * y * p;   // 2^k (atan y_k - y_k)
        // after halvings the reduced argument carries their rounding (~10 ulp
        // after four), harmless in atan x - x but not in the angle itself,
        // which then comes from the library
        return {acc + t, scale > 1.0f ? atanf(x0) : x + t};
    }
};

template <> struct AtanMx<double> {
    static constexpr double kSmall = 0.1;    // eval halves the angle from here on
    // x < kSmall: the series alone, which is what eval computes there
    static __device__ __forceinline__ AtanPair<double> small(double x)
    {
        double y = x * x;
        double p = 1.0 / 23;
        p = fma(y, p, -1.0 / 21);
        p = fma(y, p, 1.0 / 19);
        p = fma(y, p, -1.0 / 17);
        p = fma(y, p, 1.0 / 15);
        p = fma(y, p, -1.0 / 13);
        p = fma(y, p, 1.0 / 11);
        p = fma(y, p, -1.0 / 9);
        p = fma(y, p, 1.0 / 7);
        p = fma(y, p, -1.0 / 5);
        p = fma(y, p, 1.0 / 3);
        const double t = -x * y * p;
        return {t, x + t};
    }
    static __device__ __forceinline__ AtanPair<double> eval(double x)
    {
        if (x > 4.0) {
            const double a = atan(x);
            return {a - x, a};
        }
        double acc = 0.0, scale = 1.0;
        for (int i = 0; i < 4 && x >= 0.1; ++i) {
            double q = 1.0 + sqrt64(fma(x, x, 1.0));
            double iq = rcp64(q);
            acc = fma(-scale * x * x * x, iq * iq, acc);
            x *= iq;
            scale *= 2.0;
        }
        double y = x * x;
        double p = 1.0 / 23;
        p = fma(y, p, -1.0 / 21);
        p = fma(y, p, 1.0 / 19);
        p = fma(y, p, -1.0 / 17);
        p = fma(y, p, 1.0 / 15);
        p = fma(y, p, -1.0 / 13);
        p = fma(y, p, 1.0 / 11);
        p = fma(y, p, -1.0 / 9);
        p = fma(y, p, 1.0 / 7);
        p = fma(y, p, -1.0 / 5);
        p = fma(y, p, 1.0 / 3);
        const double t = -scale * x * y * p;
        return {acc + t, fma(scale, x, t)};
    }
};

// ---------------------------------------------------------------------------
// planar quadrant
// ---------------------------------------------------------------------------

// corners: 0 = (a, c), 1 = (a, d), 2 = (b, c), 3 = (b, d)
template <class T>
struct PlQuad {
    T a, b, c, d, a2, c2;
    T gu, gv, gx;          // b^2 - a^2, d^2 - c^2, gu - gv
    T s[4];                // in-plane squared radius of each corner
    T e[4], twoD[4];       // r_m - D_X = (m - j_X) + e_X;  2 D_X
    T j[4];                // j_X, an integer (exact in T: |j_X| < 2^24)
    int mfirst, mlast;     // bins touched
    T two_r0m1;            // 2 r0 - 1: (r0 + m)^2 - (r0 + m - 1)^2 = two_r0m1 + 2m
};

// FP64 per-pair setup of one planar quadrant
template <class T>
__device__ __forceinline__ void pl_setup(PlQuad<T>& q, double a, double b, double c, double d,
                                         double z2, double r0)
{
    q.a = T(a); q.b = T(b); q.c = T(c); q.d = T(d);
    q.a2 = T(a * a); q.c2 = T(c * c);
    double gu = (b - a) * (b + a), gv = (d - c) * (d + c);
    q.gu = T(gu); q.gv = T(gv); q.gx = T(gu - gv);
    const double uu[4] = {a, a, b, b}, vv[4] = {c, d, c, d};
#pragma unroll
    for (int X = 0; X < 4; ++X) {
        double s = uu[X] * uu[X] + vv[X] * vv[X];
        double D = sqrt64(z2 + s);
        double pos = D - r0;
        double jj = floor(pos + 0.5);
        q.j[X] = T(jj);
        q.e[X] = T(jj - pos);
        q.twoD[X] = T(2.0 * D);
        q.s[X] = T(s);
        if (X == 0) q.mfirst = (int)floor(pos) + 1;
        if (X == 3) q.mlast = (int)ceil(pos);
    }
    q.two_r0m1 = T(2.0 * r0 - 1.0);
}

// s_m - s_X at the edge of bin m (given as T, an exact integer): the
// difference m - j_X of two integers below 2^24 is exact in T
template <class T>
__device__ __forceinline__ T pl_qedge(const PlQuad<T>& q, int X, T m)
{
    T t = (m - q.j[X]) + q.e[X];
    return t * (t + q.twoD[X]);
}

// One arc end point moving along its line (at distance p from the origin, leg
// w along the line) between in-plane squared radii s0 and s1 = s0 + dl:
//   dw = w1 - w0 = dl / (w0 + w1),   x = tan(angle swept) = p dw / (p^2 + w0 w1),
// and, with theta(s) = acos(p / sqrt s) for the end point's angle,
//   int_{s0}^{s1} theta ds = dl theta(s1) + C,   C = s0 (atan x - x) - x w0 dw
// (C for asin(p / sqrt s) with the opposite sign), while the angle swept is
// atan x.  p = 0 or dl = 0 give C = 0 and no angle.
template <class T>
struct PlSwept {
    T C, A;
};

template <class T>
struct PlStep {
    T x, dw;
};

template <class T>
__device__ __forceinline__ PlStep<T> pl_step(T p, T dl, T w0, T w1)
{
    const T tiny = T(1e-30);
    const T dw = dl * rcp_t(fmax(w0 + w1, tiny));
    return {p * dw * rcp_t(fmax(fma(p, p, w0 * w1), tiny)), dw};
}

template <class T>
__device__ __forceinline__ PlSwept<T> pl_swept(const PlStep<T>& st, T s0, T w0, const AtanPair<T>& at)
{
    return {fma(s0, at.mx, -st.x * w0 * st.dw), at.a};
}

// Walk the bins of a planar quadrant from its first one, mfirst, to
// min(mlast, whi), handing those from wlo on to sink(m, area) (area in dr^2
// units).  A bin is cut into pieces at the corners a^2 + d^2 (the upper end
// point moves from the line u = a to v = d), b^2 + c^2 (the lower one from
// v = c to u = b) and b^2 + d^2 (the end), at most three; each piece adds
// dl Theta(s1) + (corrections of both end points) to twice the bin's area, and
// Theta is carried from piece to piece by the angles the end points sweep (in
// FP64), so no piece evaluates an inverse trigonometric function of its own.
// The walk always starts at the first bin, also when the sink wants later ones
// only (a later LDS pass, a later time tile): a walk started inside the range
// would need Theta from one atan2 of the end points, accurate to FP32 rounding,
// whose error then persists over the pair's remaining bins and leaves a step
// in f.  The piece's kind of end and its squared-radius offsets are chosen by
// selects, not branches.
template <class T, class Sink>
__device__ __forceinline__ void pl_sweep(const PlQuad<T>& q, int wlo, int whi, T wgt, Sink& sink)
{
    const int mb = q.mfirst, me = min(q.mlast, whi);
    if (mb > me || q.mlast < wlo) return;
    // state at the start of the piece: offsets Q0[X] = s0 - s_X (X = AD, BC, BD),
    // s0, the kind of start, which lines the end points are on, their legs, Theta
    T Q01 = -q.gv, Q02 = -q.gu, Q03 = -(q.gu + q.gv);
    T s0 = q.s[0], wh0 = q.c, wl0 = q.a;
    bool k0e = false, k0a = false, k0b = false;   // the piece starts at a bin edge, at corner (a, d),
                                                  // at (b, c); else at (a, c)
    bool hiS = false, loA = false;
    // Theta just above the nearest corner (a, c): 0, unless the corner is the
    // origin (the voxel's projection), where the arc is a quarter circle
    double th = (q.a > T(0) || q.c > T(0)) ? 0.0 : 0.5 * M_PI;
    int m = mb;
    T acc = T(0);
    for (int guard = 0; guard < 1 << 20; ++guard) {
        const T fm = T(m);
        T Qe[4];
#pragma unroll
        for (int X = 0; X < 4; ++X) Qe[X] = pl_qedge(q, X, fm);
        const T dlE = fma(T(2), fm, q.two_r0m1);   // from edge to edge: (r0 + m)^2 - (r0 + m - 1)^2
        // the piece ends at the next corner inside the bin, else at its outer
        // edge; every choice below is a chain of selects between values that
        // are all computed (the common case has no divergent branch)
        const bool cad = !hiS && Qe[1] > T(0), cbc = !loA && Qe[2] > T(0);
        const bool atAD = cad && (!cbc || q.gx >= T(0));
        const bool atBC = cbc && !atAD;
        const bool atBD = !cad && !cbc && Qe[3] > T(0);
        const bool edge = !cad && !cbc && !atBD;
        // Q1[X] = s1 - s_X: at a corner Y it is s_Y - s_X
        T Q10 = q.gu + q.gv, Q11 = q.gu, Q12 = q.gv, Q13 = T(0);   // at (b, d)
        Q10 = atBC ? q.gu : Q10; Q11 = atBC ? q.gx : Q11; Q12 = atBC ? T(0) : Q12; Q13 = atBC ? -q.gv : Q13;
        Q10 = atAD ? q.gv : Q10; Q11 = atAD ? T(0) : Q11; Q12 = atAD ? -q.gx : Q12; Q13 = atAD ? -q.gu : Q13;
        Q10 = edge ? Qe[0] : Q10; Q11 = edge ? Qe[1] : Q11; Q12 = edge ? Qe[2] : Q12; Q13 = edge ? Qe[3] : Q13;
        // s1 - s0 from the quantity that is exactly zero at one end
        T dlc = k0a ? Q11 : Q10;   // from a corner: its offset at s1
        dlc = k0b ? Q12 : dlc;
        T dle = atBC ? -Q02 : -Q03;   // from an edge: the corner's offset at s0, or a whole bin
        dle = atAD ? -Q01 : dle;
        dle = edge ? dlE : dle;
        const T dl = k0e ? dle : dlc;
        // legs of the end points at s1 on their current lines
        const T wh1 = sqrt_t(hiS ? Q11 + q.a2 : Q10 + q.c2);
        const T wl1 = sqrt_t(loA ? Q12 + q.c2 : Q10 + q.a2);
        const PlStep<T> sH = pl_step(hiS ? q.d : q.a, dl, wh0, wh1);
        const PlStep<T> sL = pl_step(loA ? q.b : q.c, dl, wl0, wl1);
        // atan x - x and atan x of both steps: the short series unless some
        // lane of the wave needs the angle halvings (rare: ~1 % of the pieces
        // on 50 mm geometries), decided once per wave so that the common case
        // has no divergent branch; both give the same result below kSmall
        AtanPair<T> aH, aL;
        if (__any(fmax(sH.x, sL.x) >= AtanMx<T>::kSmall)) {
            aH = AtanMx<T>::eval(sH.x);
            aL = AtanMx<T>::eval(sL.x);
        } else {
            aH = AtanMx<T>::small(sH.x);
            aL = AtanMx<T>::small(sL.x);
        }
        const PlSwept<T> H = pl_swept(sH, s0, wh0, aH);
        const PlSwept<T> Lo = pl_swept(sL, s0, wl0, aL);
        const T sh = hiS ? T(-1) : T(1), sl = loA ? T(-1) : T(1);
        th += (double)fma(sh, H.A, sl * Lo.A);
        acc += fma(dl, (T)th, fma(sh, H.C, sl * Lo.C));
        // advance
        Q01 = Q11; Q02 = Q12; Q03 = Q13;
        s0 = Q10 + q.s[0];
        k0e = edge;
        k0a = atAD;
        k0b = atBC;
        wh0 = atAD ? q.a : wh1;
        wl0 = atBC ? q.c : wl1;
        hiS = hiS || atAD;
        loA = loA || atBC;
        if (edge || atBD) {
            if (m >= wlo) sink(m, T(0.5) * wgt * acc);
            acc = T(0);
            if (atBD || m >= me) break;
            ++m;
        }
    }
}

// ---------------------------------------------------------------------------
// cylinder quadrant (FP64)
// ---------------------------------------------------------------------------

struct CyPair {
    double R, dm, mu, imu;       // radius, |R - rho|, 4 R rho, 1/mu (0 when rho = 0)
    const double2* lut;          // E~, F~ tables (lookup-table I_l only)
};

// how the cylinder's I_l is evaluated
enum : int {
    kIlExact = 0,       // Carlson, Eq. cyl_Il
    kIlTrapezoid = 1,   // chord of the level curve, Eq. trapezoid_Il
    kIlTable = 2,       // lookup tables of E~ and F~ (Sec. 4.2, LUT paragraph)
};

struct CyQuad {
    double a, b, c, d;
    double sa, ca, sb, cb;          // sin, cos of a/2 and b/2
    double Qac, Qad, Qbc, Qbd;       // squared corner distances psi(a or b) + (c or d)^2
    double psia, psib;               // psi(a), psi(b) = (R - rho)^2 + mu sin^2 of the half angle
    double sa2, cb2;                // sin^2(a/2), cos^2(b/2)
    int mfirst, mlast;
};

struct CyEdge {
    double sa, ca, da;   // alpha/2: sin, cos, Delta = sqrt(1 - nu sin^2)
    double sb, cb, db;   // beta/2
    double I;
};

// sin and cos of x in [0, pi/2] (a half angle of the folded interval [0, pi]):
// Taylor series through x^23 and x^22, whose first omitted terms are below
// 2e-18 on that range, so no argument reduction is needed
__device__ __forceinline__ void sincos_quarter(double x, double& s, double& c)
{
    const double y = x * x;
    double ps = -1.0 / 25852016738884976640000.0;              // -1/23!
    ps = fma(y, ps, 1.0 / 51090942171709440000.0);            // 1/21!
    ps = fma(y, ps, -1.0 / 121645100408832000.0);             // -1/19!
    ps = fma(y, ps, 1.0 / 355687428096000.0);                 // 1/17!
    ps = fma(y, ps, -1.0 / 1307674368000.0);                  // -1/15!
    ps = fma(y, ps, 1.0 / 6227020800.0);                      // 1/13!
    ps = fma(y, ps, -1.0 / 39916800.0);                       // -1/11!
    ps = fma(y, ps, 1.0 / 362880.0);                          // 1/9!
    ps = fma(y, ps, -1.0 / 5040.0);                           // -1/7!
    ps = fma(y, ps, 1.0 / 120.0);                             // 1/5!
    ps = fma(y, ps, -1.0 / 6.0);                              // -1/3!
    s = fma(x * y, ps, x);
    double pc = 1.0 / 1124000727777607680000.0;               // 1/22!
    pc = fma(y, pc, -1.0 / 2432902008176640000.0);            // -1/20!
    pc = fma(y, pc, 1.0 / 6402373705728000.0);                // 1/18!
    pc = fma(y, pc, -1.0 / 20922789888000.0);                 // -1/16!
    pc = fma(y, pc, 1.0 / 87178291200.0);                     // 1/14!
    pc = fma(y, pc, -1.0 / 479001600.0);                      // -1/12!
    pc = fma(y, pc, 1.0 / 3628800.0);                         // 1/10!
    pc = fma(y, pc, -1.0 / 40320.0);                          // -1/8!
    pc = fma(y, pc, 1.0 / 720.0);                             // 1/6!
    pc = fma(y, pc, -1.0 / 24.0);                             // -1/4!
    pc = fma(y, pc, 0.5);
    c = fma(-y, pc, 1.0);
}

__device__ __forceinline__ void cy_setup(CyQuad& q, const CyPair& P, double a, double b, double c,
                                         double d, double r0)
{
    q.a = a; q.b = b; q.c = c; q.d = d;
    double sa, ca, sb, cb;
    sincos_quarter(0.5 * a, sa, ca);
    sincos_quarter(0.5 * b, sb, cb);
    q.sa = sa; q.ca = ca; q.sb = sb; q.cb = cb;
    const double psia = fma(P.mu * sa, sa, P.dm * P.dm);
    const double psib = fma(P.mu * sb, sb, P.dm * P.dm);
    q.psia = psia;
    q.psib = psib;
    q.Qac = psia + c * c;
    q.Qad = psia + d * d;
    q.Qbc = psib + c * c;
    q.Qbd = psib + d * d;
    q.sa2 = sa * sa;
    q.cb2 = cb * cb;
    q.mfirst = (int)floor(sqrt64(q.Qac) - r0) + 1;   // nearest and farthest corners
    q.mlast = (int)ceil(sqrt64(q.Qbd) - r0);
}

// one end point of the level curve on the line v (Eq. alphabeta), half-angle form;
// isK = 1/sqrt(r^2 - (R - rho)^2); Qav, Qbv = psi(a or b) + v^2.  r^2 - Q is
// one fma: its error is that of the rounded Q, as for (r - sqrt Q)(r + sqrt Q)
template <int NW>
__device__ __forceinline__ void cy_endpoint(const CyQuad& q, const CyPair& P, double r, double v,
                                            double Qav, double Qbv, double isK, double& s, double& c,
                                            double& dl)
{
    double qa = fma(r, r, -Qav);                // r^2 - v^2 - psi(a)
    if (!(qa > 0.0)) {
        s = q.sa; c = q.ca;
        dl = sqrt64<NW>(fma(r, r, -q.psia)) * isK;
        return;
    }
    double qb = fma(r, r, -Qbv);                // r^2 - v^2 - psi(b)
    if (!(qb < 0.0)) {
        s = q.sb; c = q.cb;
        dl = sqrt64<NW>(fma(r, r, -q.psib)) * isK;
        return;
    }
    // sin^2 = (qa + mu sa^2) / mu and cos^2 = (mu cb^2 - qb) / mu, both > 0 here
    s = sqrt64_pos<NW>(fma(qa, P.imu, q.sa2));
    c = sqrt64_pos<NW>(fma(-qb, P.imu, q.cb2));
    dl = v * isK;
}

// E(sigma, nu) from sin, cos and Delta of sigma: E = s R_F(c^2, D^2, 1) -
// nu s^3 R_D(c^2, D^2, 1) / 3 (DLMF 19.25.9), with Carlson's duplication and
// the series of DLMF 19.36.1-2 through degree 7.  Their truncation error is
// ~eps^8 / 4 for eps = max |1 - x_i / A|, so the duplication stops once
// eps < 1/35 (relative error ~1e-13; 4e-15 measured over amplitudes to 1.55
// rad and nu sin^2 up to 0.99999) in the FP64 kernels and once eps < 1/12
// (truncation 2e-11 measured, 5e-10 with the FP32 series terms below) in the
// FP32-I/O ones (NW = 1), whose outputs round at 6e-8: that saves most lanes a
// duplication step, and on 128^3 voxels x 256 cylinders moves the signals'
// error against FP64 from 5.7e-8 to 6.9e-8 (relative L2).
// TABLE: stop at eps < 1e-4 instead (truncation far below rounding) and also
// return F = s R_F(c^2, D^2, 1).
// The duplication runs on 4^n times the n-th iterates: a step then adds
// lambda to each (no scaling), the stopping test compares 4^n A_n with the
// fixed initial deviation, and the factors 2^n that the scaling leaves on
// R_F and on the R_D series are applied once at the end.  With c^2, D^2 <= 1
// = z, z stays the largest argument, so A_D = (x + y + 3z)/5 >= A_F = (x + y
// + z)/3 and the test needs A_F only.  x and y start at c^2 + tiny and D^2 +
// tiny (tiny = 1e-300, or 1e-30 for the FP32 seeds of NW = 1, which changes
// R_F and R_D by ~1e-15 relative at most), so every square root in the loop
// has a positive argument.
template <int NW, bool TABLE = false>
__device__ __forceinline__ double ellip_e_scd(double s, double c, double dl, double nu, double* f_out = nullptr)
{
    double x = fma(c, c, Tiny<NW>::value), y = fma(dl, dl, Tiny<NW>::value), z = 1.0;
    double sx = fabs(c), sy = dl, sz = 1.0;
    double AF = (x + y + z) * (1.0 / 3.0);
    double AD = (x + y + 3.0 * z) * 0.2;
    // largest |A - x_i| over both means: z is the largest argument and A_D >= A_F
    const double dev = fmax(z - AF, AD - fmin(x, y));
    const double thr = (TABLE ? 1.0e4 : (NW == 1 ? 12.0 : 35.0)) * dev;
    const int itmax = TABLE ? 40 : 12;
    double p2 = 1.0, sumD = 0.0;
    if (thr >= AF) {
        // the first step, with z = sqrt(z) = 1
        const double lam = fma(sx, sy, sx + sy);
        z += lam;
        sumD = rcp64<NW>(z);
        x += lam;
        y += lam;
        AF += lam;
        p2 = 2.0;
        sx = sqrt64_pos<NW>(x);
        sy = sqrt64_pos<NW>(y);
        sz = sqrt64_pos<NW>(z);
#pragma unroll 1
        for (int it = 1; it < itmax && thr >= AF; ++it) {
            double lam = fma(sx, sy, fma(sx, sz, sy * sz));
            sumD = fma(p2, rcp64<NW>(sz * (z + lam)), sumD);
            x += lam;
            y += lam;
            z += lam;
            AF += lam;
            p2 *= 2.0;
            sx = sqrt64_pos<NW>(x);
            sy = sqrt64_pos<NW>(y);
            sz = sqrt64_pos<NW>(z);
        }
    }
    AD = (x + y + 3.0 * z) * 0.2;
    double rAF = rsq64<NW>(AF), iAF = rAF * rAF;
    double X = (AF - x) * iAF, Y = (AF - y) * iAF, Z = -X - Y;
    if constexpr (NW == 1) {
        // FP32-I/O kernels: the series' corrections to 1 are O(eps^2) <= ~7e-3
        // (eps < 1/12 at the stop), so FP32 (twice the FP64 rate on gfx950)
        // leaves ~5e-10 relative error on E; the deviations X, Y themselves
        // are formed in FP64
        const float xf = (float)X, yf = (float)Y, zf = -xf - yf;
        const float e2 = fmaf(xf, yf, -zf * zf), e3 = xf * yf * zf;
        const float df = fmaf(e2, fmaf(e2, fmaf(e2, -5.0f / 208.0f, 1.0f / 24.0f), -0.1f),
                              e3 * fmaf(e2, fmaf(e2, 1.0f / 16.0f, -3.0f / 44.0f), fmaf(e3, 3.0f / 104.0f, 1.0f / 14.0f)));
        const double rf = (1.0 + (double)df) * rAF * p2;
        const double rAD = rsq64<NW>(AD), iAD = rAD * rAD;
        const float xd = (float)((AD - x) * iAD), yd = (float)((AD - y) * iAD);
        const float zd = -(xd + yd) * (1.0f / 3.0f);
        const float xy = xd * yd, z2 = zd * zd;
        const float d2 = fmaf(-6.0f, z2, xy), d3 = fmaf(3.0f, xy, -8.0f * z2) * zd, d4 = 3.0f * (xy - z2) * z2,
                    d5 = xy * z2 * zd;
        float t2 = fmaf(d3, 45.0f / 272.0f, fmaf(d2, -1.0f / 16.0f, 9.0f / 88.0f));
        t2 = fmaf(d2, t2, fmaf(d3, -9.0f / 52.0f, fmaf(d4, 3.0f / 20.0f, fmaf(d5, -9.0f / 68.0f, -3.0f / 14.0f))));
        const float t3 = fmaf(d3, 3.0f / 40.0f, fmaf(d4, -9.0f / 68.0f, 1.0f / 6.0f));
        const float dd = fmaf(d2, t2, fmaf(d3, t3, fmaf(d4, -3.0f / 22.0f, d5 * (3.0f / 26.0f))));
        const double rd = fma(p2 * (1.0 + (double)dd) * iAD, rAD, 3.0 * sumD);
        if (TABLE) *f_out = s * rf;
        return s * fma(-(nu * (1.0 / 3.0)) * (s * s), rd, rf);
    }
    double E2 = fma(X, Y, -Z * Z), E3 = X * Y * Z;
    // 1 - E2/10 + E3/14 + E2^2/24 - 3 E2 E3/44 - 5 E2^3/208 + 3 E3^2/104 + E2^2 E3/16
    double sf = fma(E2, fma_vvv(E2, fma_vsv(E2, -5.0 / 208.0, 1.0 / 24.0), -0.1), 1.0);
    sf = fma(E3, fma_vvv(E2, fma_vsv(E2, 1.0 / 16.0, -3.0 / 44.0), fma_vsv(E3, 3.0 / 104.0, 1.0 / 14.0)), sf);
    double rf = sf * rAF * p2;
    double rAD = rsq64<NW>(AD), iAD = rAD * rAD;
    X = (AD - x) * iAD;
    Y = (AD - y) * iAD;
    Z = -(X + Y) * (1.0 / 3.0);
    double XY = X * Y, Z2 = Z * Z;
    double D2 = XY - 6.0 * Z2, D3 = (3.0 * XY - 8.0 * Z2) * Z, D4 = 3.0 * (XY - Z2) * Z2, D5 = XY * Z2 * Z;
    // 1 - 3 D2/14 + D3/6 + 9 D2^2/88 - 3 D4/22 - 9 D2 D3/52 + 3 D5/26 - D2^3/16 + 3 D3^2/40
    //   + 3 D2 D4/20 + 45 D2^2 D3/272 - 9 (D3 D4 + D2 D5)/68, grouped by powers of D2 and D3
    double t2 = fma(D3, 45.0 / 272.0, fma_vsv(D2, -1.0 / 16.0, 9.0 / 88.0));
    t2 = fma(D2, t2, fma(D3, -9.0 / 52.0, fma(D4, 3.0 / 20.0, fma_vsv(D5, -9.0 / 68.0, -3.0 / 14.0))));
    double t3 = fma(D3, 3.0 / 40.0, fma_vsv(D4, -9.0 / 68.0, 1.0 / 6.0));
    double ser = fma(D2, t2, fma(D3, t3, fma(D4, -3.0 / 22.0, fma(D5, 3.0 / 26.0, 1.0))));
    double rd = fma(p2 * ser * iAD, rAD, 3.0 * sumD);
    if (TABLE) *f_out = s * rf;
    return s * fma(-(nu * (1.0 / 3.0)) * (s * s), rd, rf);
}

// ---------------------------------------------------------------------------
// lookup tables of E~(s, nu) = E(arcsin s, nu) and F~(s, nu) = F(arcsin s, nu)
// ---------------------------------------------------------------------------
// Both axes use the power-law grid of Eq. LUT_sampling, x_n = top (1 - (1 -
// n/(N-1))^4), n = 0..N-1, top = 1 - 1e-16, which crowds the nodes towards the
// logarithmic singularity of F at (1, 1).  Node (s_i, nu_j) holds {E~, F~} at
// index j N + i, so the four corners of a cell are two 32-byte pairs.
constexpr double kLutTop = 1.0 - 1e-16;
constexpr double kLutInvTop = 1.0 / kLutTop;

// node x_n; n / (N - 1) as the product with the rounded reciprocal plus one
// correction step (the correctly rounded quotient)
__device__ __forceinline__ double lut_node(int n)
{
    constexpr double inv = 1.0 / (double)(kLutN - 1);
    const double dn = (double)n;
    double q = dn * inv;
    q = fma(fma(-q, (double)(kLutN - 1), dn), inv, q);
    const double t = 1.0 - q;
    return kLutTop * (1.0 - t * t * t * t);
}

// the grid cell [x_n, x_{n+1}] holding x, by the inverse of the grid map,
// t = 1 - (1 - x/top)^(1/4) (two square roots), and the weight of x in it,
// linear in the coordinate: (x - x_n) / (x_{n+1} - x_n)
template <int NW>
__device__ __forceinline__ void lut_cell(double x, int& n, double& w)
{
    const double y = fmin(fmax(x * kLutInvTop, 0.0), 1.0);
    const double p = (1.0 - sqrt64<NW>(sqrt64<NW>(1.0 - y))) * (double)(kLutN - 1);
    n = max(0, min((int)p, kLutN - 2));
    const double x0 = lut_node(n), x1 = lut_node(n + 1);
    const double d = x1 - x0;
    w = (fmin(x, kLutTop) - x0) * (NW >= 2 ? rcp64_full(d) : rcp64(d));
}

// bilinear E~ and F~ at (s, nu), nu's cell (j, wn) given
template <int NW>
__device__ __forceinline__ void lut_ef(const double2* __restrict__ T, double s, int j, double wn, double& E,
                                       double& F)
{
    int i;
    double ws;
    lut_cell<NW>(s, i, ws);
    const double2* r = T + (j * kLutN + i);
    const double2 a = r[0], b = r[1], c = r[kLutN], d = r[kLutN + 1];
    const double e0 = fma(ws, b.x - a.x, a.x), e1 = fma(ws, d.x - c.x, c.x);
    const double f0 = fma(ws, b.y - a.y, a.y), f1 = fma(ws, d.y - c.y, c.y);
    E = fma(wn, e1 - e0, e0);
    F = fma(wn, f1 - f0, f0);
}

// E(beta/2, nu) - E(alpha/2, nu) from the sines of the half angles by the
// tables: E~ directly for nu <= 1; for nu > 1 the reciprocal-modulus form
// (Eq. reciprocal_modulus) E(t, nu) = sqrt(nu) [E~(sqrt(nu) sin t, 1/nu) -
// (1 - 1/nu) F~(sqrt(nu) sin t, 1/nu)], whose first argument stays <= 1 by
// Lemma exact_integral.  Both end points share the nu cell.
template <int NW>
__device__ __forceinline__ double lut_de(const double2* __restrict__ T, double sa, double sb, double nu)
{
    const bool rec = nu > 1.0;
    const double inu = NW >= 2 ? rcp64_full(nu) : rcp64(nu);
    const double q = rec ? inu : nu;
    const double g = rec ? sqrt64<NW>(nu) : 1.0;
    const double cf = rec ? 1.0 - inu : 0.0;
    int j;
    double wn;
    lut_cell<NW>(q, j, wn);
    double Ea, Fa, Eb, Fb;
    lut_ef<NW>(T, g * sa, j, wn, Ea, Fa);
    lut_ef<NW>(T, g * sb, j, wn, Eb, Fb);
    return g * fma(-cf, Fb - Fa, Eb - Ea);
}

// asin(u) for 0 <= u <= 0.05: odd Taylor series through u^11 (the first
// omitted term is < 5e-18 relative)
__device__ __forceinline__ double asin_small(double u)
{
    double y = u * u;
    double p = 63.0 / 2816;
    p = fma(y, p, 35.0 / 1152);
    p = fma(y, p, 5.0 / 112);
    p = fma(y, p, 3.0 / 40);
    p = fma(y, p, 1.0 / 6);
    return fma(u * y, p, u);
}

// atan(t) for 0 <= t <= 1: four halvings of the angle, tan(x/2) = t / (1 +
// sqrt(1 + t^2)), take t below tan(pi/64) < 0.05, where the odd Taylor series
// through t^13 has its first omitted term below 3e-20 relative.  Its
// coefficients 1/3 .. 1/13 are taken over the common denominator 45045, so
// each is an integer that the instruction encodes as a literal.
__device__ __forceinline__ double atan_unit(double t)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) t *= rcp64_full(1.0 + sqrt64_pos(fma(t, t, 1.0)));
    const double y = t * t, y2 = y * y, y3 = y2 * y;
    const double p = 45045.0 - 15015.0 * y + 9009.0 * y2 - 6435.0 * y3 + 5005.0 * (y2 * y2) -
                     4095.0 * (y2 * y3) + 3465.0 * (y3 * y3);
    return (16.0 / 45045.0) * t * p;
}

// atan2(y, x) on the full circle from atan_unit of min/max(|x|, |y|), with
// the octant restored by reflections; 0 for x = y = 0
__device__ __forceinline__ double atan2_full(double y, double x)
{
    const double ax = fabs(x), ay = fabs(y);
    const double mn = fmin(ax, ay), mx = fmax(ax, ay);
    double a = mx > 0.0 ? atan_unit(mn * rcp64_full(mx)) : 0.0;
    if (ay > ax) a = 0.5 * M_PI - a;
    if (x < 0.0) a = M_PI - a;
    return copysign(a, y);
}

// Alg. 4 triple at the edge of radius r: half-angle state of alpha, beta and I
// (Eq. cyl_Il; the chord of the level curve, Eq. trapezoid_Il, or the tables)
template <int NW, int IL = kIlExact>
__device__ __forceinline__ void cy_edge(const CyQuad& q, const CyPair& P, double r, CyEdge& E)
{
    // K = r^2 - (R - rho)^2 = 2 R rho + b(r).  K <= 0: the shell misses the
    // surface, r^2 - v^2 - psi(a) <= 0 on both lines, so both end points clamp
    // at a (no branch of their own) and I = 0; their Delta (and 1/sqrt K) are
    // then not finite and not used
    double K = (r - P.dm) * (r + P.dm);
    double isK = rsq64<NW>(K);
    cy_endpoint<NW>(q, P, r, q.d, q.Qad, q.Qbd, isK, E.sa, E.ca, E.da);
    cy_endpoint<NW>(q, P, r, q.c, q.Qac, q.Qbc, isK, E.sb, E.cb, E.db);
    double cr = fma(E.sb, E.ca, -E.cb * E.sa);   // sin(beta/2 - alpha/2)
    if (!(cr > 0.0 && K > 0.0)) { E.I = 0.0; return; }
    if (IL == kIlTrapezoid) {
        // (beta - alpha)/2 (Psi(alpha) + Psi(beta)) with Psi = sqrt(K) Delta
        const double cs = fma(E.cb, E.ca, E.sb * E.sa);   // cos(beta/2 - alpha/2)
        const double sg = (cr <= 0.05 && cs > 0.0) ? asin_small(cr) : atan2_full(cr, cs);
        E.I = K * isK * sg * (E.da + E.db);
        return;
    }
    double nu = P.mu * isK * isK;
    if (IL == kIlTable) {
        E.I = 2.0 * K * isK * lut_de<NW>(P.lut, E.sa, E.sb, nu);
        return;
    }
    const double sbda = E.sb * E.da, sbsa = E.sb * E.sa, dd = E.db * E.da, nss = nu * sbsa;
    double den = fma(E.cb, E.cb, sbda * sbda);   // 1 - nu sin^2 sin^2
    double idn = rcp64<NW>(den);
    double ss = fma(sbda, E.ca, -E.sa * (E.cb * E.db)) * idn;
    double cs = fma(E.cb, E.ca, sbsa * dd) * idn;
    double ds = fma(nss, E.cb * E.ca, dd) * idn;
    double es = ellip_e_scd<NW>(ss, cs, ds, nu);
    E.I = 2.0 * K * isK * fma(-nss, ss, es);
}

// The steps of both end-point angles between consecutive edges (negative
// steps count as zero).  The half angles lie in [0, pi/2], so the cosine of a
// half step is >= 0, and a step whose half-step sine cr is <= 0.05 is 2 asin(cr)
// by the short series, with no division; unless every active lane of the wave
// has such steps, 2 atan2(cr, cos).
__device__ __forceinline__ void angle_steps(const CyEdge& E0, const CyEdge& E1, double& da, double& db)
{
    const double cra = fma(E1.sa, E0.ca, -E1.ca * E0.sa), crb = fma(E1.sb, E0.cb, -E1.cb * E0.sb);
    const double ua = fmax(cra, 0.0), ub = fmax(crb, 0.0);
    if (__all(fmax(ua, ub) <= 0.05)) {
        da = 2.0 * asin_small(ua);
        db = 2.0 * asin_small(ub);
        return;
    }
    const double dta = fma(E1.ca, E0.ca, E1.sa * E0.sa), dtb = fma(E1.cb, E0.cb, E1.sb * E0.sb);
    da = cra > 0.0 ? 2.0 * atan2_full(cra, dta) : 0.0;
    db = crb > 0.0 ? 2.0 * atan2_full(crb, dtb) : 0.0;
}

template <int NW, int IL, class Sink>
__device__ __forceinline__ void cy_sweep(const CyQuad& q, const CyPair& P, double r0, int wlo, int whi,
                                         double wgt, Sink& sink)
{
    const int mb = max(q.mfirst, wlo), me = min(q.mlast, whi);
    if (mb > me) return;
    const double wR = wgt * P.R;
    // Eq. area_D_l_xi, times J0 = R, between the edges Ea (inner) and Eb (outer)
    auto shell = [&](int m, const CyEdge& Ea, const CyEdge& Eb) {
        double dal, dbe;
        angle_steps(Ea, Eb, dal, dbe);
        sink(m, wR * fma(dal, q.d, fma(-q.c, dbe, Eb.I - Ea.I)));
    };
    // The inner edge of the first bin, r0 + mfirst - 1, does not pass the
    // nearest corner and the outer edge of the last one, r0 + mlast, is past
    // the farthest: there both end points sit at u = a (resp. u = b) and I = 0,
    // so these two edges are set rather than evaluated (a walk the window
    // clips evaluates its end edges).  Every lane's loop is one edge shorter.
    auto corner_edge = [](double s, double c, CyEdge& E) {
        E.sa = s; E.ca = c; E.da = 1.0;
        E.sb = s; E.cb = c; E.db = 1.0;
        E.I = 0.0;
    };
    CyEdge E0, E1;
    if (mb > q.mfirst)
        cy_edge<NW, IL>(q, P, r0 + (mb - 1), E0);
    else
        corner_edge(q.sa, q.ca, E0);
    const bool tail = me == q.mlast;
    const int mend = tail ? me - 1 : me;   // the last edge evaluated
    // two shells per trip, the edge records alternating roles (no copies)
    int m = mb;
    for (; m < mend; m += 2) {
        cy_edge<NW, IL>(q, P, r0 + m, E1);
        shell(m, E0, E1);
        cy_edge<NW, IL>(q, P, r0 + (m + 1), E0);
        shell(m + 1, E1, E0);
    }
    if (m == mend) {
        cy_edge<NW, IL>(q, P, r0 + m, E1);
        shell(m, E0, E1);
        if (tail) {
            corner_edge(q.sb, q.cb, E0);
            shell(me, E1, E0);
        }
    } else if (tail) {
        corner_edge(q.sb, q.cb, E1);
        shell(me, E0, E1);
    }
}

}  // namespace patop
