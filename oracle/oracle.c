/*
 * FP64 CPU oracle for the matrix-free photoacoustic operator A and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test-suite, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or table with the HIP library.
 *
 * It is deliberately plain and slow: it follows the paper's algorithms step by
 * step in double precision, with no blocking, fusion or reordering.
 *
 *   system kernel h        Eq. def_h / Eq. def_bh (Sec. 3.1), support as stated
 *                          after Eq. def_downsampling; g from Prop. 1 (Sec. 2.5)
 *   forward A              Alg. 1 (loop over transducers), Eq. discrete_conv,
 *                          Eq. discrete_conv_2, Eq. def_downsampling
 *   surface coefficients   Alg. 3, Eq. ui_area, bin range Eq. rmin_rmax
 *   shell area |M_i^l|     Alg. 4 (separable form, four quadrants, carried
 *                          triples alpha, beta, I), Eq. uvminmax, Eq. alphabeta,
 *                          Eq. area_D_l_xi; planar: Sec. 4.1, Eq. plane_primitive;
 *                          cylinder: Sec. 4.2, Eq. folded_intervals, Eq. cyl_Il
 *                          (Lemma exact_integral, appendix on elliptic integrals)
 *   point coefficients     Alg. 2, Eq. def_f_point, midpoint tensor rule (Prop. 2)
 *   trapezoidal I_l        Eq. trapezoid_Il (cylinder; the planar I_l stays exact)
 *   lookup-table I_l       Sec. 4.2 (LUT paragraph): E~(s, nu) = E(arcsin s, nu) and
 *                          F~(s, nu) = F(arcsin s, nu) on the power-law grid of
 *                          Eq. LUT_sampling, bilinear interpolation, nu > 1 through
 *                          the reciprocal-modulus transformation Eq. reciprocal_modulus
 *   coarse area grid       Remark 1: the area of each shell of step fine bins,
 *                          split evenly over those bins (step = 1: exact)
 *   adjoint A^T            Alg. 5, 6, 7 (transpose of the downsampling,
 *                          correlation with the reversed kernel, gather)
 *
 * Readings of points the paper leaves open (also listed in the design notes):
 *   - bins are half-open [tau_{l-1}, tau_l); the signal is the untruncated sum over
 *     every fine bin m in Z; bins that cannot reach an output sample are skipped;
 *   - arcsin(u/rho) of the planar primitive is evaluated as atan2(u, w) with the
 *     leg w = sqrt(rho^2 - u^2) taken exactly (w = v_max at an unclamped alpha,
 *     w = v_min at an unclamped beta), and the arcsin difference of Eq.
 *     plane_primitive as one atan2 of the cross and dot products of the two
 *     legs: the same function, without the loss near |u/rho| = 1;
 *   - the cylinder's Phi(v, r) = arccos(...) is evaluated through its half angle,
 *     sin^2(Phi/2) = (r^2 - v^2 - (R - rho)^2)/(4 R rho), and E(theta, nu) by
 *     Carlson's symmetric forms, E = s R_F(c^2, 1 - nu s^2, 1)
 *     - (nu/3) s^3 R_D(c^2, 1 - nu s^2, 1), valid for nu > 1 whenever
 *     nu s^2 <= 1 (guaranteed by Lemma exact_integral), so the reciprocal-modulus
 *     transformation is not needed;
 *   - R_F and R_D follow Carlson's duplication algorithm with his published
 *     stopping rule (Carlson 1995; DLMF 19.36.1, 19.36.2).
 *
 * Transducers are packed as 16 doubles: shape, c0[3], e1[3], e2[3], half_w,
 * half_h, radius, theta_max, half_len, unused.  Units are SI.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PLANAR 0
#define OR_CYLINDER 1
#define OR_MODE_SURFACE 0
#define OR_MODE_POINT 1
#define OR_MODE_TRAPEZOID 2
#define OR_MODE_LUT 3

/* ------------------------------------------------------------------------- */
/* Carlson symmetric elliptic integrals (DLMF 19.36.1 and 19.36.2)            */
/* ------------------------------------------------------------------------- */

double or_carlson_rf(double x, double y, double z)
{
    const double r = 1e-16;
    double A0 = (x + y + z) / 3.0;
    double Q = pow(3.0 * r, -1.0 / 6.0) *
               fmax(fabs(A0 - x), fmax(fabs(A0 - y), fabs(A0 - z)));
    double A = A0, p4 = 1.0;
    for (int it = 0; it < 200 && p4 * Q >= fabs(A); ++it) {
        double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        double lam = sx * sy + sx * sz + sy * sz;
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
        A = 0.25 * (A + lam);
        p4 *= 0.25;
    }
    /* X = (A0 - x0)/(4^n A_n) = (A_n - x_n)/A_n */
    double X = (A - x) / A, Y = (A - y) / A, Z = -X - Y;
    double E2 = X * Y - Z * Z, E3 = X * Y * Z;
    return (1.0 - E2 / 10.0 + E3 / 14.0 + E2 * E2 / 24.0 - 3.0 * E2 * E3 / 44.0) / sqrt(A);
}

double or_carlson_rd(double x, double y, double z)
{
    const double r = 1e-16;
    double A0 = (x + y + 3.0 * z) / 5.0;
    double Q = pow(0.25 * r, -1.0 / 6.0) *
               fmax(fabs(A0 - x), fmax(fabs(A0 - y), fabs(A0 - z)));
    double A = A0, p4 = 1.0, sum = 0.0;
    for (int it = 0; it < 200 && p4 * Q >= fabs(A); ++it) {
        double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        double lam = sx * sy + sx * sz + sy * sz;
        sum += p4 / (sz * (z + lam));
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
        A = 0.25 * (A + lam);
        p4 *= 0.25;
    }
    double X = (A - x) / A, Y = (A - y) / A, Z = -(X + Y) / 3.0;
    double XY = X * Y, Z2 = Z * Z;
    double E2 = XY - 6.0 * Z2;
    double E3 = (3.0 * XY - 8.0 * Z2) * Z;
    double E4 = 3.0 * (XY - Z2) * Z2;
    double E5 = XY * Z2 * Z;
    double ser = 1.0 - 3.0 * E2 / 14.0 + E3 / 6.0 + 9.0 * E2 * E2 / 88.0 - 3.0 * E4 / 22.0
               - 9.0 * E2 * E3 / 52.0 + 3.0 * E5 / 26.0;
    return p4 * ser / (A * sqrt(A)) + 3.0 * sum;
}

/* E(phi, m) = int_0^phi sqrt(1 - m sin^2 t) dt from sin(phi), cos(phi), for
   0 <= phi <= pi/2 and m sin^2(phi) <= 1 (m may exceed 1). */
static double ellip_e_sc(double s, double c, double m)
{
    double x = c * c, y = 1.0 - m * s * s;
    if (y < 0.0) y = 0.0;
    if (s == 0.0) return 0.0;
    if (x == 0.0 && y == 0.0) return s;   /* phi = pi/2, m = 1: E = 1 */
    return s * or_carlson_rf(x, y, 1.0) - (m / 3.0) * s * s * s * or_carlson_rd(x, y, 1.0);
}

double or_ellip_e(double phi, double m)
{
    return ellip_e_sc(sin(phi), cos(phi), m);
}

double or_ellip_f(double phi, double m)
{
    double s = sin(phi), c = cos(phi);
    double y = 1.0 - m * s * s;
    if (y < 0.0) y = 0.0;
    return s * or_carlson_rf(c * c, y, 1.0);
}

/* ------------------------------------------------------------------------- */
/* Lookup tables of E~ and F~ (Sec. 4.2, LUT paragraph)                       */
/* ------------------------------------------------------------------------- */

/* Both axes use the grid of Eq. LUT_sampling, x_n = (1 - eps)[1 - (1 - t_n)^4],
   t_n = (n - 1)/(N - 1), n = 1..N, eps = 1e-16; here indices run from 0.  The
   table holds, for every node (s_i, nu_j), the pair E~, F~ at
   tab[2 (j N + i)] and tab[2 (j N + i) + 1], in double precision like every
   other array of the method. */
static const double lut_eps = 1e-16;
static int lut_size = 1000;
static int lut_built = 0;
static double* lut_tab = NULL;

static double lut_node(int n, int N)
{
    double t = 1.0 - (double)n / (N - 1);
    return (1.0 - lut_eps) * (1.0 - t * t * t * t);
}

static void lut_build(void)
{
    int N = lut_size;
    free(lut_tab);
    lut_tab = (double*)malloc(sizeof(double) * 2 * (size_t)N * N);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < N; ++j) {
        double nu = lut_node(j, N);
        for (int i = 0; i < N; ++i) {
            double s = lut_node(i, N);
            double c2 = (1.0 - s) * (1.0 + s);   /* cos^2(arcsin s) */
            double y = 1.0 - nu * s * s;
            double e = 0.0, f = 0.0;
            if (s > 0.0) {
                double rf = or_carlson_rf(c2, y, 1.0);
                f = s * rf;
                e = f - (nu / 3.0) * s * s * s * or_carlson_rd(c2, y, 1.0);
            }
            lut_tab[2 * ((size_t)j * N + i)] = e;
            lut_tab[2 * ((size_t)j * N + i) + 1] = f;
        }
    }
    lut_built = 1;
}

static void lut_ensure(void)
{
    if (!lut_built) lut_build();
}

/* table size per axis (tests only; the method uses 1000) */
void or_lut_set_size(int n)
{
    if (n >= 2 && n != lut_size) {
        lut_size = n;
        lut_built = 0;
    }
}

/* the cell [x_n, x_{n+1}] of the grid holding x, found by inverting Eq.
   LUT_sampling, t = 1 - (1 - x/(1 - eps))^(1/4) (two square roots), and the
   linear weight of x in that cell, (x - x_n)/(x_{n+1} - x_n) */
static void lut_locate(double x, int N, int* n, double* w)
{
    double y = x / (1.0 - lut_eps);
    if (y > 1.0) y = 1.0;
    if (y < 0.0) y = 0.0;
    double t = 1.0 - sqrt(sqrt(1.0 - y));
    int k = (int)floor(t * (N - 1));
    if (k > N - 2) k = N - 2;
    double x0 = lut_node(k, N), x1 = lut_node(k + 1, N);
    *n = k;
    *w = (fmin(x, 1.0 - lut_eps) - x0) / (x1 - x0);
}

/* bilinear interpolation of E~ and F~ at (s, nu) in [0, 1]^2 */
static void lut_interp(double s, double nu, double* E, double* F)
{
    int N = lut_size, i, j;
    double ws, wn;
    lut_locate(s, N, &i, &ws);
    lut_locate(nu, N, &j, &wn);
    double e = 0.0, f = 0.0;
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
            double wt = (di ? ws : 1.0 - ws) * (dj ? wn : 1.0 - wn);
            const double* t = lut_tab + 2 * ((size_t)(j + dj) * N + (i + di));
            e += wt * t[0];
            f += wt * t[1];
        }
    *E = e;
    *F = f;
}

/* E(theta, nu) for theta in [0, pi/2] with nu sin^2(theta) <= 1, from s =
   sin(theta), by the tables: E~(s, nu) when nu <= 1, otherwise Eq.
   reciprocal_modulus, E = sqrt(nu) [E~(sqrt(nu) s, 1/nu) - (1 - 1/nu) F~(sqrt(nu) s, 1/nu)]
   (arcsin(sqrt(nu) s) is the amplitude the tables are indexed by through its sine) */
static double lut_e(double s, double nu)
{
    double E, F;
    if (nu <= 1.0) {
        lut_interp(s, nu, &E, &F);
        return E;
    }
    double sq = sqrt(nu);
    lut_interp(sq * s, 1.0 / nu, &E, &F);
    return sq * (E - (1.0 - 1.0 / nu) * F);
}

/* for tests: E(theta, nu) by the tables, from s = sin(theta) */
double or_lut_e(double s, double nu)
{
    lut_ensure();
    return lut_e(s, nu);
}

/* for tests: the table entries at node (i, j) and the node coordinates */
void or_lut_entry(int i, int j, double* s, double* nu, double* E, double* F)
{
    lut_ensure();
    *s = lut_node(i, lut_size);
    *nu = lut_node(j, lut_size);
    *E = lut_tab[2 * ((size_t)j * lut_size + i)];
    *F = lut_tab[2 * ((size_t)j * lut_size + i) + 1];
}

/* ------------------------------------------------------------------------- */
/* Gauss-Legendre nodes (Newton iteration on the Legendre recurrence)         */
/* ------------------------------------------------------------------------- */

#define GL_MAX 32
static void gauss_legendre(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ------------------------------------------------------------------------- */
/* System kernel h (Eq. def_h, Eq. def_bh; g from Prop. 1)                     */
/* ------------------------------------------------------------------------- */

typedef struct {
    int phi_type;          /* 0 cone, 1 Wendland (1 - r/kappa)^2 */
    double kappa, c;
    int eir_kind;          /* 0 Gaussian-windowed cosine, 1 sampled */
    double fc, sig, tc, te;
    const double* smp;
    long nsmp;
    double dt;
} kspec;

static double phi_eval(const kspec* K, double r)
{
    if (r >= K->kappa) return 0.0;
    double t = 1.0 - r / K->kappa;
    return K->phi_type == 0 ? t : t * t;
}

/* g(t) = -1/2 c t phi(c |t|)   (Prop. 1) */
static double g_eval(const kspec* K, double t)
{
    return -0.5 * K->c * t * phi_eval(K, K->c * fabs(t));
}

static double e_eval(const kspec* K, double t)
{
    if (K->eir_kind == 0) {
        if (t < 0.0 || t > K->te) return 0.0;
        double d = t - K->tc;
        return cos(2.0 * M_PI * K->fc * d) * exp(-d * d / (2.0 * K->sig * K->sig));
    }
    if (t < 0.0) return 0.0;
    double u = t / K->dt;
    long j = (long)floor(u);
    if (j >= K->nsmp - 1) return (j == K->nsmp - 1 && u == (double)j) ? K->smp[j] : 0.0;
    double a = u - j;
    return (1.0 - a) * K->smp[j] + a * K->smp[j + 1];
}

static int cmp_dbl(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* (g * Lambda)(x) = int_{-D}^{D} (1 - |s|/D) g(x + s) ds, piecewise polynomial:
   split at the breakpoints of both factors, Gauss-Legendre on each piece. */
static double g_tri(const kspec* K, double x, double D, const double* gx, const double* gw, int ng)
{
    double bp[8];
    int nb = 0;
    double a = K->kappa / K->c;
    double cand[6] = {-D, 0.0, D, -x, -x - a, -x + a};
    for (int i = 0; i < 6; ++i)
        if (cand[i] >= -D && cand[i] <= D) bp[nb++] = cand[i];
    qsort(bp, nb, sizeof(double), cmp_dbl);
    double acc = 0.0;
    for (int p = 0; p + 1 < nb; ++p) {
        double lo = bp[p], hi = bp[p + 1];
        if (hi <= lo) continue;
        double hm = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
        for (int q = 0; q < ng; ++q) {
            double s = mid + hm * gx[q];
            acc += hm * gw[q] * (1.0 - fabs(s) / D) * g_eval(K, x + s);
        }
    }
    return acc;
}

/* h[n] = int e(t') (g * Lambda)(n D - t') dt'  (Eq. def_bh rewritten with the
   triangle Lambda(s) = max(0, 1 - |s|/D), D = 1/(U fs)). */
int or_build_kernel(int phi_type, double kappa, int eir_kind, const double* eir_par,
                    const double* eir_samples, long n_samples, double eir_dt,
                    double c, double fs, int U, double* h, long cap, long* n_first, long* len)
{
    kspec K;
    memset(&K, 0, sizeof K);
    K.phi_type = phi_type;
    K.kappa = kappa;
    K.c = c;
    K.eir_kind = eir_kind;
    double te;
    if (eir_kind == 0) {
        K.fc = eir_par[0]; K.sig = eir_par[1]; K.tc = eir_par[2]; K.te = eir_par[3];
        te = K.te;
    } else {
        K.smp = eir_samples; K.nsmp = n_samples; K.dt = eir_dt;
        te = (n_samples - 1) * eir_dt;
    }
    double D = 1.0 / (U * fs);
    double a = kappa / c;
    long nf = (long)floor(-a / D) - 1;
    long nl = (long)ceil((a + te) / D) + 1;
    long n = nl - nf + 1;
    *n_first = nf;
    *len = n;
    if (n > cap) return -1;

    double ix[8], iw[8], ox[20], ow[20];
    gauss_legendre(8, ix, iw);
    gauss_legendre(20, ox, ow);

    long nbmax = 16 + (eir_kind == 1 ? n_samples : 0);
    double* bp = (double*)malloc(sizeof(double) * nbmax);
    for (long j = 0; j < n; ++j) {
        double tn = (nf + j) * D;
        double lo = fmax(0.0, tn - a - D), hi = fmin(te, tn + a + D);
        h[j] = 0.0;
        if (hi <= lo) continue;
        int nb = 0;
        double offs[9] = {0.0, D, -D, a, -a, a + D, a - D, -a + D, -a - D};
        for (int i = 0; i < 9; ++i) {
            double t = tn - offs[i];
            if (t > lo && t < hi) bp[nb++] = t;
        }
        if (eir_kind == 1) {
            long j0 = (long)ceil(lo / eir_dt), j1 = (long)floor(hi / eir_dt);
            for (long q = j0; q <= j1; ++q) {
                double t = q * eir_dt;
                if (t > lo && t < hi) bp[nb++] = t;
            }
        }
        bp[nb++] = lo;
        bp[nb++] = hi;
        qsort(bp, nb, sizeof(double), cmp_dbl);
        double acc = 0.0;
        for (int p = 0; p + 1 < nb; ++p) {
            double l0 = bp[p], l1 = bp[p + 1];
            if (l1 <= l0) continue;
            int sub = 1 + (int)((l1 - l0) / (0.02 / (eir_kind == 0 ? K.fc : 1.0 / eir_dt)));
            double step = (l1 - l0) / sub;
            for (int s = 0; s < sub; ++s) {
                double p0 = l0 + s * step, hm = 0.5 * step, mid = p0 + hm;
                for (int q = 0; q < 20; ++q) {
                    double t = mid + hm * ox[q];
                    acc += hm * ow[q] * e_eval(&K, t) * g_tri(&K, tn - t, D, ix, iw, 8);
                }
            }
        }
        h[j] = acc;
    }
    free(bp);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Separable geometry: quadrants of D after reflection (Eq. uvminmax)          */
/* ------------------------------------------------------------------------- */

typedef struct {
    double a, b, c, d;   /* u in [a, b], v in [c, d], all >= 0 */
} oquad;

typedef struct {
    int shape, nq;
    oquad q[4];
    double z2;           /* planar: x_i[3]^2 */
    double R, rho;       /* cylinder */
    double J0;
    double rmin, rmax;
} opair;

static double wrap_pi(double u)
{
    /* into (-pi, pi] */
    while (u <= -M_PI) u += 2.0 * M_PI;
    while (u > M_PI) u -= 2.0 * M_PI;
    return u;
}

static double psi_of(const opair* P, double u)
{
    if (P->shape == OR_PLANAR) return u * u + P->z2;
    double sh = sin(0.5 * u);
    double d = P->R - P->rho;
    return d * d + 4.0 * P->R * P->rho * sh * sh;
}

static void pair_setup(const double* tr, const double* x, opair* P)
{
    int shape = (int)tr[0];
    const double *c0 = tr + 1, *e1 = tr + 4, *e2 = tr + 7;
    double n3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                    e1[0] * e2[1] - e1[1] * e2[0]};
    double d[3] = {x[0] - c0[0], x[1] - c0[1], x[2] - c0[2]};
    double ua[2][2];     /* up to two u-intervals */
    int nu = 0;
    double v1, v2;
    P->shape = shape;
    if (shape == OR_PLANAR) {
        /* frame (e1, e2, e1 x e2) centred at c0 (Sec. 4.1) */
        double x1 = d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2];
        double x2 = d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2];
        double x3 = d[0] * n3[0] + d[1] * n3[1] + d[2] * n3[2];
        double L1 = tr[10], L2 = tr[11];
        double u1 = -L1 - x1, u2 = L1 - x1;
        v1 = -L2 - x2;
        v2 = L2 - x2;
        P->z2 = x3 * x3;
        P->J0 = 1.0;
        /* Eq. uvminmax */
        ua[0][0] = fmax(u1, 0.0); ua[0][1] = fmax(u2, 0.0);
        ua[1][0] = fmax(-u2, 0.0); ua[1][1] = fmax(-u1, 0.0);
        nu = 2;
    } else {
        /* frame (e2, e1 x e2, e1) centred at c0 (Sec. 4.2) */
        double x1 = d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2];
        double x2 = d[0] * n3[0] + d[1] * n3[1] + d[2] * n3[2];
        double x3 = d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2];
        double R = tr[12], th = tr[13], Lz = tr[14];
        P->R = R;
        P->rho = sqrt(x1 * x1 + x2 * x2);
        /* focal line (Sec. 4.2): rho at rounding level (below 1e-10 R) is the
           rho = 0 case, whose angle atan2 would take from rounding noise */
        if (P->rho <= 1e-10 * R) P->rho = 0.0;
        P->J0 = R;
        double thi = P->rho > 0.0 ? atan2(x2, x1) : 0.0;
        double u1 = wrap_pi(-th - thi), u2 = wrap_pi(th - thi);
        v1 = -Lz - x3;
        v2 = Lz - x3;
        /* Eq. folded_intervals */
        if (u1 < 0.0 && 0.0 < u2) {
            ua[0][0] = 0.0; ua[0][1] = -u1; ua[1][0] = 0.0; ua[1][1] = u2; nu = 2;
        } else if (u2 < u1) {
            ua[0][0] = u1; ua[0][1] = M_PI; ua[1][0] = -u2; ua[1][1] = M_PI; nu = 2;
        } else if (0.0 <= u1) {
            ua[0][0] = u1; ua[0][1] = u2; nu = 1;
        } else {
            ua[0][0] = -u2; ua[0][1] = -u1; nu = 1;
        }
    }
    double va[2][2] = {{fmax(v1, 0.0), fmax(v2, 0.0)}, {fmax(-v2, 0.0), fmax(-v1, 0.0)}};
    P->nq = 0;
    P->rmin = INFINITY;
    P->rmax = 0.0;
    for (int i = 0; i < nu; ++i)
        for (int j = 0; j < 2; ++j) {
            if (!(ua[i][1] > ua[i][0]) || !(va[j][1] > va[j][0])) continue;
            oquad* q = &P->q[P->nq++];
            q->a = ua[i][0]; q->b = ua[i][1]; q->c = va[j][0]; q->d = va[j][1];
            /* Eq. closedform_rminrmax */
            double rlo = sqrt(psi_of(P, q->a) + q->c * q->c);
            double rhi = sqrt(psi_of(P, q->b) + q->d * q->d);
            if (rlo < P->rmin) P->rmin = rlo;
            if (rhi > P->rmax) P->rmax = rhi;
        }
}

/* triple carried by Alg. 4 for one quadrant at one edge */
typedef struct { double al, be, I; } otriple;

/* alpha/beta = clamped Phi(v, r) (Eq. alphabeta) and I (Eq. plane_primitive /
   Eq. cyl_Il) for one quadrant at radius r. */
static otriple quad_edge(const opair* P, const oquad* q, double r, int mode)
{
    otriple T;
    double r2 = r * r;
    if (P->shape == OR_PLANAR) {
        double rho2 = r2 - P->z2;
        double wa, wb;
        /* alpha = Phi^(v_max, r) */
        double qa = rho2 - q->d * q->d, qb = rho2 - q->c * q->c;
        if (qa <= q->a * q->a) { T.al = q->a; wa = sqrt(fmax(0.0, rho2 - q->a * q->a)); }
        else if (qa >= q->b * q->b) { T.al = q->b; wa = sqrt(fmax(0.0, rho2 - q->b * q->b)); }
        else { T.al = sqrt(qa); wa = q->d; }
        if (qb <= q->a * q->a) { T.be = q->a; wb = sqrt(fmax(0.0, rho2 - q->a * q->a)); }
        else if (qb >= q->b * q->b) { T.be = q->b; wb = sqrt(fmax(0.0, rho2 - q->b * q->b)); }
        else { T.be = sqrt(qb); wb = q->c; }
        if (!(T.be > T.al)) { T.I = 0.0; return T; }
        /* I = 1/2 [u sqrt(rho^2 - u^2) + rho^2 arcsin(u/rho)]_alpha^beta */
        double ang = atan2(T.be * wa - T.al * wb, wa * wb + T.al * T.be);
        T.I = 0.5 * ((T.be * wb - T.al * wa) + rho2 * ang);
        return T;
    }
    /* cylinder */
    double R = P->R, rho = P->rho;
    double dm = R - rho, dp = R + rho;
    double pa = psi_of(P, q->a), pb = psi_of(P, q->b);
    double sa, ca, sb, cb;       /* sin, cos of alpha/2 and beta/2 */
    double qa = r2 - q->d * q->d, qb = r2 - q->c * q->c;
    int ia = 0, ib = 0;          /* end point inside (a, b): on the line v = d, resp. v = c */
    if (qa <= pa) { T.al = q->a; sa = sin(0.5 * q->a); ca = cos(0.5 * q->a); }
    else if (qa >= pb) { T.al = q->b; sa = sin(0.5 * q->b); ca = cos(0.5 * q->b); }
    else {
        double h = atan2(sqrt(qa - dm * dm), sqrt(dp * dp - qa));
        T.al = 2.0 * h; sa = sin(h); ca = cos(h); ia = 1;
    }
    if (qb <= pa) { T.be = q->a; sb = sin(0.5 * q->a); cb = cos(0.5 * q->a); }
    else if (qb >= pb) { T.be = q->b; sb = sin(0.5 * q->b); cb = cos(0.5 * q->b); }
    else {
        double h = atan2(sqrt(qb - dm * dm), sqrt(dp * dp - qb));
        T.be = 2.0 * h; sb = sin(h); cb = cos(h); ib = 1;
    }
    double Kc = r2 - dm * dm;   /* 2 R rho + b(r) */
    if (!(T.be > T.al) || !(Kc > 0.0)) { T.I = 0.0; return T; }
    if (mode == OR_MODE_TRAPEZOID) {
        /* Eq. trapezoid_Il: the level curve u -> Psi(u, r) = sqrt(r^2 - psi(u))
           replaced by the chord between its end points.  An end point inside
           (a, b) lies on its line by definition (Eq. alphabeta), so Psi there
           is that line's v; only a clamped end point needs the square root */
        double pa_ = ia ? q->d : sqrt(fmax(0.0, r2 - psi_of(P, T.al)));
        double pb_ = ib ? q->c : sqrt(fmax(0.0, r2 - psi_of(P, T.be)));
        T.I = 0.5 * (T.be - T.al) * (pa_ + pb_);
        return T;
    }
    double nu = 4.0 * R * rho / Kc;
    if (mode == OR_MODE_LUT)
        T.I = 2.0 * sqrt(Kc) * (lut_e(sb, nu) - lut_e(sa, nu));
    else
        T.I = 2.0 * sqrt(Kc) * (ellip_e_sc(sb, cb, nu) - ellip_e_sc(sa, ca, nu));
    return T;
}

/* |D^l| summed over quadrants (Eq. area_D_l_xi, Eq. swept_u) given the triples at
   the previous edge; updates the triples to the new edge (Alg. 4). */
static double alg4_step(const opair* P, otriple* tri, double r, int mode)
{
    double area = 0.0;
    for (int k = 0; k < P->nq; ++k) {
        const oquad* q = &P->q[k];
        otriple T = quad_edge(P, q, r, mode);
        area += P->J0 * ((T.al - tri[k].al) * q->d + T.I - tri[k].I - (T.be - tri[k].be) * q->c);
        tri[k] = T;
    }
    return area;
}

static void alg4_init(const opair* P, otriple* tri)
{
    for (int k = 0; k < P->nq; ++k) {
        tri[k].al = P->q[k].a;
        tri[k].be = P->q[k].a;
        tri[k].I = 0.0;
    }
}

/* Area of {x in Sigma : r0 <= |x - x_i| < r1} by Alg. 4 (single shell). */
double or_shell_area(const double* tr, const double* x, double r0, double r1)
{
    opair P;
    pair_setup(tr, x, &P);
    otriple tri[4];
    for (int k = 0; k < P.nq; ++k) tri[k] = quad_edge(&P, &P.q[k], r0, 0);
    return alg4_step(&P, tri, r1, 0);
}

/* Bin range (Eq. rmin_rmax) and the areas of every bin in it, carrying the
   triples from edge to edge (Alg. 3 + Alg. 4).  Returns the count, or -1. */
static long pair_areas(const double* tr, const double* x, double c, double t0, double ufs, int mode,
                       long* lmin, long* lmax, double* out, long cap)
{
    opair P;
    pair_setup(tr, x, &P);
    if (P.nq == 0) { *lmin = 1; *lmax = 0; return 0; }
    long l0 = (long)floor((P.rmin / c - t0) * ufs) + 1;
    long l1 = (long)ceil((P.rmax / c - t0) * ufs);
    *lmin = l0;
    *lmax = l1;
    if (l1 - l0 + 1 > cap) return -1;
    otriple tri[4];
    alg4_init(&P, tri);
    for (long l = l0; l <= l1; ++l) out[l - l0] = alg4_step(&P, tri, c * (t0 + l / ufs), mode);
    return l1 - l0 + 1;
}

long or_pair_areas(const double* tr, const double* x, double c, double t0, double ufs,
                   long* lmin, long* lmax, double* out, long cap)
{
    return pair_areas(tr, x, c, t0, ufs, 0, lmin, lmax, out, cap);
}

static long floor_div(long a, long b)
{
    long q = a / b;
    return (q * b > a) ? q - 1 : q;
}

/* Remark 1: the area of each shell of `step` fine bins, shell j holding the bins
   (j - 1) step + 1 .. j step, split evenly over its bins.  a holds the fine areas
   of the bins *l0 .. *l0 + cnt - 1; on return out holds the split areas of the
   bins *l0 .. *l0 + (returned count) - 1, whole shells.  Returns -1 if more than
   cap bins. */
static long shell_split(int step, long* l0, long cnt, const double* a, double* out, long cap)
{
    if (cnt <= 0) return cnt;
    long b0 = *l0, b1 = *l0 + cnt - 1;
    long j0 = -floor_div(-b0, step), j1 = -floor_div(-b1, step);   /* ceil(b / step) */
    long s0 = (j0 - 1) * step + 1, s1 = j1 * step;
    if (s1 - s0 + 1 > cap) return -1;
    for (long j = j0; j <= j1; ++j) {
        double sum = 0.0;
        for (long l = (j - 1) * step + 1; l <= j * step; ++l)
            if (l >= b0 && l <= b1) sum += a[l - b0];
        for (long l = (j - 1) * step + 1; l <= j * step; ++l) out[l - s0] = sum / step;
    }
    *l0 = s0;
    return s1 - s0 + 1;
}

/* The areas a surface method uses for one pair: exact (mode 0), with the
   trapezoidal I_l (mode 2) or the lookup-table I_l (mode 3), on the fine bins
   (step 1) or split from the shells of the coarse area grid (step > 1).  The
   tables must exist (lut_ensure) before a mode-3 call. */
static long pair_areas_mode(const double* tr, const double* x, double c, double t0, double ufs, int mode,
                            int step, long* lmin, long* lmax, double* out, long cap)
{
    long cnt = pair_areas(tr, x, c, t0, ufs, mode, lmin, lmax, out, cap);
    if (cnt <= 0 || step <= 1) return cnt;
    double* fine = (double*)malloc(sizeof(double) * cnt);
    memcpy(fine, out, sizeof(double) * cnt);
    long n = shell_split(step, lmin, cnt, fine, out, cap);
    free(fine);
    if (n >= 0) *lmax = *lmin + n - 1;
    return n;
}

long or_pair_areas_mode(const double* tr, const double* x, double c, double t0, double ufs, int mode,
                        int step, long* lmin, long* lmax, double* out, long cap)
{
    if (mode == OR_MODE_LUT) lut_ensure();
    return pair_areas_mode(tr, x, c, t0, ufs, mode, step, lmin, lmax, out, cap);
}

/* ------------------------------------------------------------------------- */
/* Quadrature points (midpoint tensor rule on D, barycentres of the cells)     */
/* ------------------------------------------------------------------------- */

void or_quad_points(const double* tr, int n1, int n2, double* pts, double* dA)
{
    const double *c0 = tr + 1, *e1 = tr + 4, *e2 = tr + 7;
    double n3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                    e1[0] * e2[1] - e1[1] * e2[0]};
    if ((int)tr[0] == OR_PLANAR) {
        double L1 = tr[10], L2 = tr[11];
        *dA = (2.0 * L1 / n1) * (2.0 * L2 / n2);
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n2; ++b) {
                double u = -L1 + (a + 0.5) * (2.0 * L1 / n1);
                double v = -L2 + (b + 0.5) * (2.0 * L2 / n2);
                double* p = pts + 3 * (a * n2 + b);
                for (int k = 0; k < 3; ++k) p[k] = c0[k] + u * e1[k] + v * e2[k];
            }
    } else {
        double R = tr[12], th = tr[13], Lz = tr[14];
        *dA = R * (2.0 * th / n1) * (2.0 * Lz / n2);
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n2; ++b) {
                double t = -th + (a + 0.5) * (2.0 * th / n1);
                double z = -Lz + (b + 0.5) * (2.0 * Lz / n2);
                double* p = pts + 3 * (a * n2 + b);
                for (int k = 0; k < 3; ++k)
                    p[k] = c0[k] + R * cos(t) * e2[k] + R * sin(t) * n3[k] + z * e1[k];
            }
    }
}

int or_num_threads(void);

/* ------------------------------------------------------------------------- */
/* Operator                                                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    const double* tr;
    int K;
    long n[3];
    double origin[3], w;
    const double* h;
    long nf, hlen;
    double c, fs, t0;
    int L, U, mode, q1, q2, step;
    long Mlo, Mhi;     /* fine bins that can reach an output sample */
} oop;

static void op_init(oop* o, const double* tr, int K, const long* n, const double* origin, double w,
                    const double* h, long nf, long hlen, double c, double fs, double t0,
                    int L, int U, int mode, int q1, int q2, int step)
{
    o->tr = tr; o->K = K; o->step = step < 1 ? 1 : step;
    for (int a = 0; a < 3; ++a) { o->n[a] = n[a]; o->origin[a] = origin[a]; }
    o->w = w; o->h = h; o->nf = nf; o->hlen = hlen;
    o->c = c; o->fs = fs; o->t0 = t0; o->L = L; o->U = U; o->mode = mode; o->q1 = q1; o->q2 = q2;
    long nl = nf + hlen - 1;
    if (mode == OR_MODE_LUT) lut_ensure();
    o->Mlo = 1 - nl;
    o->Mhi = (long)U * L - nf;
}

static void voxel_xyz(const oop* o, long i, double* x)
{
    long ix = i % o->n[0], iy = (i / o->n[0]) % o->n[1], iz = i / (o->n[0] * o->n[1]);
    x[0] = o->origin[0] + ix * o->w;
    x[1] = o->origin[1] + iy * o->w;
    x[2] = o->origin[2] + iz * o->w;
}

/* geometric coefficients f_k on bins [Mlo, Mhi] (Alg. 3 or Alg. 2), B volumes */
static void fcoef_range(const oop* o, int k, const double* coef, int B, long N, long i0, long i1,
                        double* f /* B x M, accumulated */)
{
    long M = o->Mhi - o->Mlo + 1;
    const double* tr = o->tr + 16 * (long)k;
    double ufs = o->U * o->fs;
    double* tmp = NULL;
    long cap = 1 << 16;
    double *pts = NULL, dA = 0.0;
    int Q = o->q1 * o->q2;
    if (o->mode != OR_MODE_POINT) tmp = (double*)malloc(sizeof(double) * cap);
    else {
        pts = (double*)malloc(sizeof(double) * 3 * Q);
        or_quad_points(tr, o->q1, o->q2, pts, &dA);
    }
    for (long i = i0; i < i1; ++i) {
        int any = 0;
        for (int b = 0; b < B; ++b) any |= coef[b * N + i] != 0.0;
        if (!any) continue;
        double x[3];
        voxel_xyz(o, i, x);
        if (o->mode != OR_MODE_POINT) {
            long l0, l1;
            long cnt = pair_areas_mode(tr, x, o->c, o->t0, ufs, o->mode, o->step, &l0, &l1, tmp, cap);
            for (long j = 0; j < cnt; ++j) {
                long l = l0 + j;
                if (l < o->Mlo || l > o->Mhi) continue;
                double tm = o->t0 + (l - 0.5) / ufs;   /* tau_{l-1/2} */
                for (int b = 0; b < B; ++b)
                    f[b * M + (l - o->Mlo)] += coef[b * N + i] * tmp[j] / (o->c * tm);
            }
        } else {
            for (int j = 0; j < Q; ++j) {
                const double* q = pts + 3 * j;
                double r = sqrt((q[0] - x[0]) * (q[0] - x[0]) + (q[1] - x[1]) * (q[1] - x[1]) +
                                (q[2] - x[2]) * (q[2] - x[2]));
                long l = (long)floor((r / o->c - o->t0) * ufs) + 1;
                if (l < o->Mlo || l > o->Mhi) continue;
                for (int b = 0; b < B; ++b) f[b * M + (l - o->Mlo)] += coef[b * N + i] * dA / r;
            }
        }
    }
    free(tmp);
    free(pts);
}

/* geometric coefficients f_k on bins [Mlo, Mhi] (Alg. 3 or Alg. 2), B volumes;
   when `par` is set the voxel loop is shared by the OpenMP threads (each keeps
   its own partial f, summed at the end) */
static void fcoef(const oop* o, int k, const double* coef, int B, long N, double* f, int par)
{
    long M = o->Mhi - o->Mlo + 1;
    double ufs = o->U * o->fs;
    memset(f, 0, sizeof(double) * M * B);
    if (!par) {
        fcoef_range(o, k, coef, B, N, 0, N, f);
    } else {
#pragma omp parallel
        {
            double* loc = (double*)calloc((size_t)M * B, sizeof(double));
            int nt = 1, id = 0;
#ifdef _OPENMP
            nt = omp_get_num_threads();
            id = omp_get_thread_num();
#endif
            long chunk = (N + nt - 1) / nt;
            long a = id * chunk, b = a + chunk < N ? a + chunk : N;
            if (a < b) fcoef_range(o, k, coef, B, N, a, b, loc);
#pragma omp critical
            for (long j = 0; j < M * B; ++j) f[j] += loc[j];
            free(loc);
        }
    }
    for (long j = 0; j < M * B; ++j) f[j] *= ufs;
}

/* s_hat[l] = 1/U sum_{l'=1..U} (h * f)[U(l-1) + l'], l = 1..L (Eq. discrete_conv) */
static void conv_down(const oop* o, const double* f, double* s)
{
    long M = o->Mhi - o->Mlo + 1;
    for (int l = 1; l <= o->L; ++l) {
        double acc = 0.0;
        for (int lp = 1; lp <= o->U; ++lp) {
            long l2 = (long)o->U * (l - 1) + lp;
            for (long j = 0; j < o->hlen; ++j) {
                long m = l2 - (o->nf + j);
                if (m < o->Mlo || m > o->Mhi) continue;
                acc += o->h[j] * f[m - o->Mlo];
            }
        }
        (void)M;
        s[l - 1] = acc / o->U;
    }
}

/* f-coefficients of one transducer, for tests (B x M, bins Mlo..Mhi) */
void or_fcoef(const double* tr, int K, const long* n, const double* origin, double w,
              const double* h, long nf, long hlen, double c, double fs, double t0,
              int L, int U, int mode, int q1, int q2, int step, const double* coef, int B,
              int k, double* f, long* Mlo, long* Mhi)
{
    oop o;
    op_init(&o, tr, K, n, origin, w, h, nf, hlen, c, fs, t0, L, U, mode, q1, q2, step);
    *Mlo = o.Mlo;
    *Mhi = o.Mhi;
    if (f) fcoef(&o, k, coef, B, n[0] * n[1] * n[2], f, 0);
}

/* Forward operator on a subset of transducers (Alg. 1).  out is B x nk x L. */
void or_forward(const double* tr, int K, const long* n, const double* origin, double w,
                const double* h, long nf, long hlen, double c, double fs, double t0,
                int L, int U, int mode, int q1, int q2, int step, const double* coef, int B,
                const int* ksub, int nk, double* out)
{
    oop o;
    op_init(&o, tr, K, n, origin, w, h, nf, hlen, c, fs, t0, L, U, mode, q1, q2, step);
    long N = n[0] * n[1] * n[2];
    long M = o.Mhi - o.Mlo + 1;
    if (nk >= or_num_threads()) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int kk = 0; kk < nk; ++kk) {
            double* f = (double*)malloc(sizeof(double) * M * B);
            fcoef(&o, ksub[kk], coef, B, N, f, 0);
            for (int b = 0; b < B; ++b) conv_down(&o, f + b * M, out + ((long)b * nk + kk) * L);
            free(f);
        }
    } else {
        double* f = (double*)malloc(sizeof(double) * M * B);
        for (int kk = 0; kk < nk; ++kk) {
            fcoef(&o, ksub[kk], coef, B, N, f, 1);
            for (int b = 0; b < B; ++b) conv_down(&o, f + b * M, out + ((long)b * nk + kk) * L);
        }
        free(f);
    }
}

/* v_k = h^- * (up-sampling transpose of y_k) on bins Mlo..Mhi (Alg. 5) */
static void adj_prep(const oop* o, const double* yk, double* v)
{
    long M = o->Mhi - o->Mlo + 1;
    long UL = (long)o->U * o->L;
    for (long m = o->Mlo; m <= o->Mhi; ++m) {
        double acc = 0.0;
        /* (h^- * v_up)[m] = sum_j h[j - m] v_up[j],  v_up[U(l-1)+l'] = y[l]/U */
        for (long j = 0; j < o->hlen; ++j) {
            long jj = o->nf + j + m;      /* index into v_up with h index nf + j = jj - m */
            if (jj < 1 || jj > UL) continue;
            long l = (jj - 1) / o->U + 1;
            acc += o->h[j] * yk[l - 1] / o->U;
        }
        v[m - o->Mlo] = acc;
    }
    (void)M;
}

/* Adjoint on a subset of voxels (Alg. 5 with Alg. 7 or Alg. 6).
   y is B x K x L; out is B x nv. */
void or_adjoint(const double* tr, int K, const long* n, const double* origin, double w,
                const double* h, long nf, long hlen, double c, double fs, double t0,
                int L, int U, int mode, int q1, int q2, int step, const double* y, int B,
                const long* vsub, long nv, double* out)
{
    oop o;
    op_init(&o, tr, K, n, origin, w, h, nf, hlen, c, fs, t0, L, U, mode, q1, q2, step);
    long M = o.Mhi - o.Mlo + 1;
    double ufs = U * fs;
    double* V = (double*)malloc(sizeof(double) * M * K * B);
#pragma omp parallel for schedule(static)
    for (long kb = 0; kb < (long)K * B; ++kb) {
        int b = (int)(kb / K), k = (int)(kb % K);
        adj_prep(&o, y + ((long)b * K + k) * L, V + kb * M);
    }
    int Q = q1 * q2;
    double* pts = NULL;
    double* dAs = NULL;
    if (mode == OR_MODE_POINT) {
        pts = (double*)malloc(sizeof(double) * 3 * Q * K);
        dAs = (double*)malloc(sizeof(double) * K);
        for (int k = 0; k < K; ++k) or_quad_points(tr + 16 * k, q1, q2, pts + 3L * Q * k, dAs + k);
    }
#pragma omp parallel
    {
        long cap = 1 << 16;
        double* tmp = (double*)malloc(sizeof(double) * cap);
        double* z = (double*)malloc(sizeof(double) * B);
#pragma omp for schedule(dynamic, 16)
        for (long ii = 0; ii < nv; ++ii) {
            double x[3];
            voxel_xyz(&o, vsub[ii], x);
            for (int b = 0; b < B; ++b) z[b] = 0.0;
            for (int k = 0; k < K; ++k) {
                const double* t = tr + 16 * k;
                if (mode != OR_MODE_POINT) {
                    long l0, l1;
                    long cnt = pair_areas_mode(t, x, c, t0, ufs, mode, o.step, &l0, &l1, tmp, cap);
                    for (long j = 0; j < cnt; ++j) {
                        long l = l0 + j;
                        if (l < o.Mlo || l > o.Mhi) continue;
                        double tm = t0 + (l - 0.5) / ufs;
                        for (int b = 0; b < B; ++b)
                            z[b] += tmp[j] * V[((long)b * K + k) * M + (l - o.Mlo)] / (c * tm);
                    }
                } else {
                    const double* P = pts + 3L * Q * k;
                    for (int j = 0; j < Q; ++j) {
                        const double* q = P + 3 * j;
                        double r = sqrt((q[0] - x[0]) * (q[0] - x[0]) + (q[1] - x[1]) * (q[1] - x[1]) +
                                        (q[2] - x[2]) * (q[2] - x[2]));
                        long l = (long)floor((r / c - t0) * ufs) + 1;
                        if (l < o.Mlo || l > o.Mhi) continue;
                        for (int b = 0; b < B; ++b)
                            z[b] += dAs[k] * V[((long)b * K + k) * M + (l - o.Mlo)] / r;
                    }
                }
            }
            for (int b = 0; b < B; ++b) out[(long)b * nv + ii] = ufs * z[b];
        }
        free(tmp);
        free(z);
    }
    free(V);
    free(pts);
    free(dAs);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
