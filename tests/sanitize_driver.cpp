// Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
// the FP64 oracle (oracle/oracle.c, test infrastructure) and the library's
// host-only parts (the system-kernel builder and the geometry validation),
// driven through their normal entry points on small inputs, including the
// argument and geometry errors the library must reject.  Built and run by
// tests/test_sanitizers.py; exits non-zero on the first wrong result, and the
// sanitizers abort on the first memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "patop.h"

extern "C" {
double or_carlson_rf(double x, double y, double z);
double or_carlson_rd(double x, double y, double z);
double or_ellip_e(double phi, double m);
double or_lut_e(double s, double nu);
void or_lut_set_size(int n);
int or_build_kernel(int phi_type, double kappa, int eir_kind, const double* eir_par, const double* eir_samples,
                    long n_samples, double eir_dt, double c, double fs, int U, double* h, long cap, long* n_first,
                    long* len);
long or_pair_areas_mode(const double* tr, const double* x, double c, double t0, double ufs, int mode, int step,
                        long* lmin, long* lmax, double* out, long cap);
void or_quad_points(const double* tr, int n1, int n2, double* pts, double* dA);
void or_forward(const double* tr, int K, const long* n, const double* origin, double w, const double* h, long nf,
                long hlen, double c, double fs, double t0, int L, int U, int mode, int q1, int q2, int step,
                const double* coef, int B, const int* ksub, int nk, double* out);
void or_adjoint(const double* tr, int K, const long* n, const double* origin, double w, const double* h, long nf,
                long hlen, double c, double fs, double t0, int L, int U, int mode, int q1, int q2, int step,
                const double* y, int B, const long* vsub, long nv, double* out);
void or_set_threads(int n);
}

static int failures = 0;

#define CHECK(cond)                                                                \
    do {                                                                           \
        if (!(cond)) {                                                             \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                            \
        }                                                                          \
    } while (0)

// packed transducer rows: shape, c0[3], e1[3], e2[3], half_w, half_h, R, theta_max, L_z, pad
static void planar_row(double* r, double z)
{
    std::memset(r, 0, 16 * sizeof(double));
    r[0] = 0; r[3] = z; r[4] = 1; r[8] = 1; r[10] = 0.5e-3; r[11] = 0.4e-3;
}
static void cylinder_row(double* r, double x)
{
    std::memset(r, 0, 16 * sizeof(double));
    r[0] = 1; r[1] = x - 6e-3; r[6] = 1; r[7] = 1; r[12] = 6e-3; r[13] = 0.3; r[14] = 1e-3;
}

int main()
{
    or_set_threads(2);
    // elliptic integrals
    // R_F(x, x, x) = x^(-1/2), R_D(x, x, x) = x^(-3/2), E(phi, 0) = phi, E(phi, 1) = sin(phi)
    CHECK(std::fabs(or_carlson_rf(2.5, 2.5, 2.5) - 1.0 / std::sqrt(2.5)) < 1e-15);
    CHECK(std::fabs(or_carlson_rd(0.5, 0.5, 0.5) - std::pow(0.5, -1.5)) < 1e-14);
    CHECK(std::fabs(or_ellip_e(0.7, 0.0) - 0.7) < 1e-15);
    CHECK(std::fabs(or_ellip_e(0.7, 1.0) - std::sin(0.7)) < 1e-15);
    or_lut_set_size(64);
    CHECK(std::fabs(or_lut_e(0.5, 0.3) - or_ellip_e(std::asin(0.5), 0.3)) < 1e-3);

    // system kernel, both builders
    const double eir[4] = {5e6, 0.12493e-6, 0.6246e-6, 1.2493e-6};
    std::vector<double> h(4096);
    long nf = 0, len = 0;
    CHECK(or_build_kernel(1, 0.15e-3, 0, eir, nullptr, 0, 0.0, 1500.0, 40e6, 2, h.data(), (long)h.size(), &nf,
                          &len) == 0);
    CHECK(len > 0 && len < 4096);
    pat_eir e{};
    e.kind = PAT_EIR_GAUSS_COS;
    e.fc = eir[0]; e.sigma_t = eir[1]; e.t_c = eir[2]; e.t_e = eir[3];
    std::vector<double> h2(4096);
    int64_t nf2 = 0, len2 = 0;
    CHECK(pat_build_kernel(PAT_PHI_WENDLAND2, 0.15e-3, &e, 1500.0, 40e6, 2, h2.data(), 4096, &nf2, &len2) ==
          PAT_OK);
    CHECK(nf2 == nf && len2 == len);
    double hmax = 0.0, dmax = 0.0;
    for (long i = 0; i < len; ++i) {
        hmax = std::fmax(hmax, std::fabs(h[i]));
        dmax = std::fmax(dmax, std::fabs(h[i] - h2[i]));
    }
    CHECK(dmax < 1e-12 * hmax);
    CHECK(pat_build_kernel(PAT_PHI_CONE, 0.15e-3, &e, 1500.0, 40e6, 2, h2.data(), 3, &nf2, &len2) == PAT_E_ARG);
    CHECK(pat_build_kernel(PAT_PHI_CONE, 0.15e-3, nullptr, 1500.0, 40e6, 2, h2.data(), 4096, &nf2, &len2) ==
          PAT_E_ARG);

    // areas of one pair in every surface mode, quadrature points
    double pl[16], cy[16];
    planar_row(pl, 6e-3);
    cylinder_row(cy, 5e-3);
    const double x[3] = {0.1e-3, -0.05e-3, 0.2e-3};
    std::vector<double> out(1 << 14);
    for (int mode : {0, 2, 3})
        for (int step : {1, 3})
            for (const double* tr : {pl, cy}) {
                long l0 = 0, l1 = 0;
                long cnt = or_pair_areas_mode(tr, x, 1500.0, 2e-6, 120e6, mode, step, &l0, &l1, out.data(),
                                              (long)out.size());
                CHECK(cnt > 0 && l1 - l0 + 1 == cnt);
            }
    std::vector<double> pts(3 * 12);
    double dA = 0.0;
    or_quad_points(cy, 4, 3, pts.data(), &dA);
    CHECK(std::fabs(12 * dA - 2 * 0.3 * 6e-3 * 2e-3) < 1e-18);

    // operator and its transpose on a 4^3 grid, two transducers, both methods
    double tr[32];
    std::memcpy(tr, pl, sizeof pl);
    std::memcpy(tr + 16, cy, sizeof cy);
    const long n[3] = {4, 4, 4};
    const double origin[3] = {-0.15e-3, -0.15e-3, -0.15e-3};
    const int L = 120;
    std::vector<double> coef(64), y(2 * L), s(2 * L), z(64);
    for (int i = 0; i < 64; ++i) coef[i] = 0.01 * (i % 7);
    for (int i = 0; i < 2 * L; ++i) y[i] = std::sin(0.1 * i);
    const int ks[2] = {0, 1};
    std::vector<long> vs(64);
    for (int i = 0; i < 64; ++i) vs[i] = i;
    for (int mode : {0, 1}) {
        or_forward(tr, 2, n, origin, 0.1e-3, h.data(), nf, len, 1500.0, 40e6, 2.5e-6, L, 2, mode, 3, 3, 1,
                   coef.data(), 1, ks, 2, s.data());
        or_adjoint(tr, 2, n, origin, 0.1e-3, h.data(), nf, len, 1500.0, 40e6, 2.5e-6, L, 2, mode, 3, 3, 1,
                   y.data(), 1, vs.data(), 64, z.data());
        double lhs = 0.0, rhs = 0.0, ns = 0.0, ny = 0.0;
        for (int i = 0; i < 2 * L; ++i) { lhs += s[i] * y[i]; ns += s[i] * s[i]; ny += y[i] * y[i]; }
        for (int i = 0; i < 64; ++i) rhs += coef[i] * z[i];
        CHECK(ns > 0.0 && std::fabs(lhs - rhs) <= 1e-12 * std::sqrt(ns * ny));
    }

    // geometry validation of the library
    pat_transducer t[2];
    std::memset(t, 0, sizeof t);
    t[0].shape = PAT_PLANAR;
    t[0].c0[2] = 6e-3; t[0].e1[0] = 1; t[0].e2[1] = 1; t[0].half_w = 0.5e-3; t[0].half_h = 0.4e-3;
    t[1].shape = PAT_CYLINDER;
    t[1].c0[0] = -1e-3; t[1].e1[2] = 1; t[1].e2[0] = 1; t[1].radius = 6e-3; t[1].theta_max = 0.3;
    t[1].half_len = 1e-3;
    pat_grid g{};
    for (int a = 0; a < 3; ++a) { g.n[a] = 4; g.origin[a] = -0.15e-3; }
    g.spacing = 0.1e-3;
    double dlow = 0.0;
    CHECK(pat_check_geometry(t, 2, &g, 0.15e-3, &dlow) == PAT_OK && dlow > 0.15e-3);
    CHECK(pat_check_geometry(t, 2, &g, 0.15e-3, nullptr) == PAT_OK);
    CHECK(pat_check_geometry(nullptr, 2, &g, 0.15e-3, &dlow) == PAT_E_ARG);
    CHECK(pat_check_geometry(t, 0, &g, 0.15e-3, &dlow) == PAT_E_ARG);
    CHECK(pat_check_geometry(t, 2, &g, 50e-3, &dlow) == PAT_E_SEPARATION);
    pat_transducer bad = t[1];
    bad.e2[0] = 0.9;
    CHECK(pat_check_geometry(&bad, 1, &g, 0.15e-3, &dlow) == PAT_E_FRAME);
    bad = t[1];
    bad.theta_max = 2.0;
    CHECK(pat_check_geometry(&bad, 1, &g, 0.15e-3, &dlow) == PAT_E_SHAPE);
    bad = t[0];
    bad.c0[1] = NAN;
    CHECK(pat_check_geometry(&bad, 1, &g, 0.15e-3, &dlow) == PAT_E_ARG);
    pat_grid gz = g;
    gz.n[2] = 0;
    CHECK(pat_check_geometry(t, 2, &gz, 0.15e-3, &dlow) == PAT_E_ARG);

    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("sanitized host checks passed\n");
    return 0;
}
