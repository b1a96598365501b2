// Internal types shared by the host side (host.hip) and the device kernels
// (kernels.hip) of the patop library.  Not part of the ABI.
//
// Every length on the device is expressed in units of the area step
// da = step * dr, dr = c / (U fs) the fine radial step: area shell j (fine bins
// (j - 1) step + 1 .. j step of the paper's [tau_{m-1}, tau_m)) is then the
// radial interval [r0 + j - 1, r0 + j) with r0 = c t0 / da.  With step = 1 (and
// always for the quadrature) shells are the fine bins.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace patop {

constexpr int kThreads = 256;      // work-group size (4 wave64)
constexpr int kBrickX = 8;         // voxel brick owned by one work-group, one voxel per thread
constexpr int kBrickY = 8;
constexpr int kBrickZ = 4;
static_assert(kBrickX * kBrickY * kBrickZ == kThreads, "one voxel per thread");
static_assert(kBrickX == 8 && kBrickY == 8 && kBrickZ == 4, "four 4 x 4 x 4 wave sub-cubes per brick");
constexpr int kHistQuad = 1024;    // quadrature kernels: bins per pass and volume (their windows
                                   // are narrow and more of them fit a CU with 8 KB each)
constexpr int kMaxNB = 8;          // volumes per launch
constexpr int kLutN = 1000;        // nodes per axis of the E~ / F~ tables (lookup-table I_l)

// One transducer, device side (all lengths in dr units).
struct TrDev {
    double base[3];     // frame coordinates (x1, x2, x3) of voxel (0,0,0)
    double g[3][3];     // g[a][d]: change of frame coordinate a per unit step of index d
    double cen[3];      // centre of the bounding sphere, global coordinates
    double rad;         // bounding-sphere radius
    double p[3];        // planar: L1, L2, -;  cylinder: R, theta_max, L_z
    double cth, sth;    // cylinder: cos and sin of theta_max
    int32_t shape;
    int32_t pad;
};

// Launch parameters (passed by value).
struct KParams {
    const TrDev* tr;
    const int32_t* kperm;   // transducer indices of this launch's shape group
    int32_t nk;             // entries of kperm
    int32_t kchunk;         // transducers per work-group
    int32_t K;              // all transducers (row stride of f / W / signals)
    int64_t n[3];
    double origin[3];       // global position of voxel (0,0,0)
    double w;               // voxel spacing
    double r0;              // c t0 / dr
    int64_t Mlo, Mcount;    // kept fine bins [Mlo, Mlo + Mcount)
    int32_t step;           // fine bins per area shell (coarse area grid; 1 = exact)
    int64_t Jlo, Jhi;       // shells that hold a kept fine bin (= Mlo, Mlo + Mcount - 1 when step = 1)
    int32_t nbx, nby, nbz;  // bricks per axis
    int32_t B;              // volumes in this launch (<= kMaxNB)
    int64_t N;
    // support of the coefficients (forward restricted to nonzero voxels)
    const int32_t* sup_list;    // voxel indices, brick by brick
    const int32_t* sup_total;   // [1] number of entries
    // lookup-table I_l: {E~, F~} on the power-law grid, node (i, j) at j N + i
    const double2* lut;
    // quadrature
    const double* qpts;     // [K][Q][3] global point coordinates
    const double* qdA;      // [K] cell area (dr^2 units)
    int32_t Q;
};

}  // namespace patop
