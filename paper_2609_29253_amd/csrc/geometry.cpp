// Host-only geometry of the patop library: bounding spheres of the
// transducer surfaces and the validation of pat_check_geometry (frames,
// shapes, and the separation of Assumption 1(iii) on a lower bound of the
// voxel-to-surface distance).  Plain C++ (no HIP).
#include <algorithm>
#include <cmath>

#include "geometry.h"

namespace patop {
namespace geom {

double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// bounding sphere of a transducer surface
void bounding_sphere(const pat_transducer& t, double cen[3], double& rad)
{
    if (t.shape == PAT_PLANAR) {
        for (int a = 0; a < 3; ++a) cen[a] = t.c0[a];
        rad = std::hypot(t.half_w, t.half_h);
    } else {
        for (int a = 0; a < 3; ++a) cen[a] = t.c0[a] + t.radius * t.e2[a];
        rad = std::hypot(2.0 * t.radius * std::sin(0.5 * t.theta_max), t.half_len);
    }
}

void grid_box(const pat_grid& g, double lo[3], double hi[3])
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = g.origin[a];
        hi[a] = g.origin[a] + (g.n[a] - 1) * g.spacing;
    }
}

static bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }


}  // namespace geom
}  // namespace patop

using namespace patop::geom;

extern "C" pat_status pat_check_geometry(const pat_transducer* tr, int32_t K, const pat_grid* grid, double kappa,
                              double* dist_lower)
{
    if (!tr || !grid || K < 1 || !(kappa > 0.0)) return PAT_E_ARG;
    for (int a = 0; a < 3; ++a)
        if (grid->n[a] < 1) return PAT_E_ARG;
    if (!(grid->spacing > 0.0) || !finite3(grid->origin)) return PAT_E_ARG;
    double lo[3], hi[3];
    grid_box(*grid, lo, hi);
    double dmin = INFINITY;
    for (int k = 0; k < K; ++k) {
        const pat_transducer& t = tr[k];
        if (t.shape != PAT_PLANAR && t.shape != PAT_CYLINDER) return PAT_E_ARG;
        if (!finite3(t.c0) || !finite3(t.e1) || !finite3(t.e2)) return PAT_E_ARG;
        if (std::fabs(dot3(t.e1, t.e1) - 1.0) > 1e-9 || std::fabs(dot3(t.e2, t.e2) - 1.0) > 1e-9 ||
            std::fabs(dot3(t.e1, t.e2)) > 1e-9)
            return PAT_E_FRAME;
        if (t.shape == PAT_PLANAR) {
            if (!(t.half_w > 0.0) || !(t.half_h > 0.0) || !std::isfinite(t.half_w) || !std::isfinite(t.half_h))
                return PAT_E_SHAPE;
        } else {
            if (!(t.radius > 0.0) || !(t.theta_max > 0.0) || !(t.theta_max < 0.5 * M_PI) || !(t.half_len > 0.0) ||
                !std::isfinite(t.radius) || !std::isfinite(t.half_len))
                return PAT_E_SHAPE;
        }
        double cen[3], rad;
        bounding_sphere(t, cen, rad);
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double o = std::max(0.0, std::max(lo[a] - cen[a], cen[a] - hi[a]));
            d2 += o * o;
        }
        dmin = std::min(dmin, std::sqrt(d2) - rad);
    }
    if (dist_lower) *dist_lower = dmin;
    // Assumption 1(iii): dist_min >= kappa (checked on a lower bound of dist_min)
    if (!(dmin >= kappa)) return PAT_E_SEPARATION;
    return PAT_OK;
}
