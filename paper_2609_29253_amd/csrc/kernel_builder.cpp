// Discrete system kernel h[n] (Eq. def_h, Eq. def_bh), host FP64.
//
//   g(t)  = -1/2 c t phi(c |t|)                         (Prop. 1)
//   h(t)  = (e * g)(t) = int g(tau) e(t - tau) dtau     (Eq. def_h)
//   h[n]  = U fs int_0^D int_0^D h(t - t' + n D) dt dt',  D = 1/(U fs)   (Eq. def_bh)
//         = int_{-D}^{D} (1 - |s|/D) h(n D + s) ds
//
// The support of h[n] is n in [-kappa U fs / c - 1, (kappa/c + T_e) U fs + 1]
// (stated after Eq. def_downsampling).  Both integrals are evaluated by
// composite Gauss-Legendre quadrature split at every point where the integrand
// loses smoothness (the kinks of phi at 0 and kappa, the ends of the EIR
// support, the samples of a sampled EIR, the apex of the triangle), so each
// piece is integrated to rounding level.
#include <algorithm>
#include <cmath>
#include <vector>

#include "patop.h"

namespace {

struct GL {
    std::vector<double> x, w;
    explicit GL(int n) : x(n), w(n)
    {
        // Newton iteration on P_n from Tricomi's estimate of the roots.
        for (int i = 0; i < n; ++i) {
            double z = std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
            double dp = 1.0;
            for (int it = 0; it < 64; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (p0 - z * p1) / (1.0 - z * z);
                double step = p1 / dp;
                z -= step;
                if (std::fabs(step) < 1e-17) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

struct Spec {
    int phi;
    double kappa, c;
    pat_eir e;
    double te;
};

double phi_of(const Spec& S, double r)
{
    if (r >= S.kappa) return 0.0;
    double t = 1.0 - r / S.kappa;
    return S.phi == PAT_PHI_CONE ? t : t * t;
}

double g_of(const Spec& S, double t) { return -0.5 * S.c * t * phi_of(S, S.c * std::fabs(t)); }

double e_of(const Spec& S, double t)
{
    if (S.e.kind == PAT_EIR_GAUSS_COS) {
        if (t < 0.0 || t > S.e.t_e) return 0.0;
        double d = t - S.e.t_c;
        return std::cos(2.0 * M_PI * S.e.fc * d) * std::exp(-0.5 * d * d / (S.e.sigma_t * S.e.sigma_t));
    }
    if (t < 0.0) return 0.0;
    double u = t / S.e.dt;
    int64_t j = (int64_t)std::floor(u);
    if (j > S.e.n_samples - 1) return 0.0;
    if (j == S.e.n_samples - 1) return u == (double)j ? S.e.samples[j] : 0.0;
    double a = u - j;
    return (1.0 - a) * S.e.samples[j] + a * S.e.samples[j + 1];
}

// breakpoints of the EIR inside [lo, hi]
void eir_breaks(const Spec& S, double lo, double hi, std::vector<double>& out)
{
    if (S.e.kind == PAT_EIR_GAUSS_COS) {
        for (double b : {0.0, S.e.t_e})
            if (b > lo && b < hi) out.push_back(b);
        return;
    }
    int64_t j0 = (int64_t)std::ceil(lo / S.e.dt), j1 = (int64_t)std::floor(hi / S.e.dt);
    for (int64_t j = std::max<int64_t>(j0, 0); j <= std::min<int64_t>(j1, S.e.n_samples - 1); ++j) {
        double b = j * S.e.dt;
        if (b > lo && b < hi) out.push_back(b);
    }
}

double max_piece(const Spec& S)
{
    // keep pieces shorter than a tenth of a carrier period (smooth EIR) or one sample
    if (S.e.kind == PAT_EIR_GAUSS_COS) return 0.1 / S.e.fc;
    return S.e.dt;
}

template <class Fn>
double integrate_pieces(std::vector<double>& bp, const GL& gl, double hmax, Fn&& f)
{
    std::sort(bp.begin(), bp.end());
    double acc = 0.0;
    for (size_t p = 0; p + 1 < bp.size(); ++p) {
        double lo = bp[p], hi = bp[p + 1];
        if (!(hi > lo)) continue;
        int sub = 1 + (int)((hi - lo) / hmax);
        double step = (hi - lo) / sub;
        for (int s = 0; s < sub; ++s) {
            double a = lo + s * step, hm = 0.5 * step, mid = a + hm;
            for (size_t q = 0; q < gl.x.size(); ++q) acc += hm * gl.w[q] * f(mid + hm * gl.x[q]);
        }
    }
    return acc;
}

// h(t) = int_{-kappa/c}^{kappa/c} g(tau) e(t - tau) dtau
double h_cont(const Spec& S, const GL& gl, double t)
{
    double a = S.kappa / S.c;
    double lo = std::max(-a, t - S.te), hi = std::min(a, t);
    if (!(hi > lo)) return 0.0;
    std::vector<double> bp{lo, hi};
    if (0.0 > lo && 0.0 < hi) bp.push_back(0.0);
    // tau where t - tau hits a breakpoint of e
    std::vector<double> eb;
    eir_breaks(S, t - hi, t - lo, eb);
    for (double b : eb) bp.push_back(t - b);
    return integrate_pieces(bp, gl, max_piece(S), [&](double tau) { return g_of(S, tau) * e_of(S, t - tau); });
}

}  // namespace

extern "C" pat_status pat_build_kernel(int32_t phi_type, double kappa, const pat_eir* eir,
                                       double sound_speed, double fs, int32_t U, double* h_out,
                                       int64_t cap, int64_t* n_first, int64_t* len)
{
    if (!eir || !n_first || !len || !(kappa > 0.0) || !(sound_speed > 0.0) || !(fs > 0.0) || U < 1)
        return PAT_E_ARG;
    if (phi_type != PAT_PHI_CONE && phi_type != PAT_PHI_WENDLAND2) return PAT_E_ARG;
    Spec S{phi_type, kappa, sound_speed, *eir, 0.0};
    if (eir->kind == PAT_EIR_GAUSS_COS) {
        if (!(eir->t_e > 0.0) || !(eir->sigma_t > 0.0) || !(eir->fc >= 0.0)) return PAT_E_ARG;
        S.te = eir->t_e;
    } else if (eir->kind == PAT_EIR_SAMPLED) {
        if (!eir->samples || eir->n_samples < 2 || !(eir->dt > 0.0)) return PAT_E_ARG;
        S.te = (eir->n_samples - 1) * eir->dt;
    } else {
        return PAT_E_ARG;
    }
    const double D = 1.0 / (U * fs), a = kappa / sound_speed;
    const int64_t nf = (int64_t)std::floor(-a / D) - 1;
    const int64_t nl = (int64_t)std::ceil((a + S.te) / D) + 1;
    *n_first = nf;
    *len = nl - nf + 1;
    if (!h_out || *len > cap) return PAT_E_ARG;

    GL inner(16), outer(16);
    // the continuous h has kinks where a kink of g meets a jump or kink of e
    std::vector<double> hk;
    {
        std::vector<double> eb;
        eir_breaks(S, -1.0, S.te + 1.0, eb);
        eb.push_back(0.0);
        eb.push_back(S.te);
        for (double b : eb)
            for (double gk : {-a, 0.0, a}) hk.push_back(b + gk);
    }
    for (int64_t n = nf; n <= nl; ++n) {
        double tn = n * D;
        std::vector<double> bp{-D, 0.0, D};
        for (double k : hk)
            if (k - tn > -D && k - tn < D) bp.push_back(k - tn);
        double v = integrate_pieces(bp, outer, D, [&](double s) {
            return (1.0 - std::fabs(s) / D) * h_cont(S, inner, tn + s);
        });
        if (!std::isfinite(v)) return PAT_E_KERNEL;
        h_out[n - nf] = v;
    }
    return PAT_OK;
}
