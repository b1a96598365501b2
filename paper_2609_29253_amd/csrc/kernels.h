// Launch plan handed from the host side to the kernel launchers.  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include "patop_internal.h"

namespace patop {

struct ShapeGroup {
    int shape;              // 0 planar, 1 cylinder
    const int32_t* kperm;   // device array of transducer indices
    int nk;
    int kchunk_fwd, kchunk_adj;
    const int32_t* items;   // (transducer, time tile) forward: items kk ntiles + t, largest estimated cost
    int nitems;             // first (nk ntiles of them); null when that forward is off
};

struct LaunchPlan {
    KParams base;           // geometry, window and table pointers (kperm/nk/kchunk/B per launch)
    ShapeGroup groups[2];
    int ngroups;
    int nbricks;
    int mode;               // 0 closed form, 1 quadrature, 2 / 3 closed form with the trapezoidal /
                            // lookup-table cylinder I_l
    bool fp64;
    int U, L;
    int jlo, jcnt;          // polyphase filter G[j], j = jlo .. jlo + jcnt - 1
    const double* G;        // [jcnt] FP64 in both variants: the zero-mean kernel amplifies any
                            // rounding of its taps by |h||f|/|h*f| (20-300) in the signal
    const double* scale;    // [Mcount]
    double* f;              // [max_batch][K][Mcount] forward workspace
    void* W;                // [max_batch][K][Mcount] adjoint workspace (float or double)
    double* z64;            // [max_batch][N] adjoint FP64 partial sums
    int32_t* sup_list;      // [N] support of the coefficients (sparse forward)
    int32_t* sup_cnt;       // [nbricks] nonzero voxels per brick (in sup_order)
    int32_t* sup_off;       // [nbricks + 1] their exclusive prefix sums (last entry: total)
    const int32_t* sup_order;   // [nbricks] brick indices in Morton order (the list's brick order)
    int tile, ntiles;       // (transducer, time tile) forward: shells per tile and tiles per transducer
                            // (tile = 0: the cube forward)
    int ncubes;             // 4 x 4 x 4 voxel cubes (one-wave work-groups of the closed-form forward and adjoint)
};

hipError_t launch_forward(const LaunchPlan& L, const void* coef, void* sig, int B, hipStream_t s);
// A restricted to the voxels where some volume's coefficient is nonzero (same result)
hipError_t launch_forward_sparse(const LaunchPlan& L, const void* coef, void* sig, int B, hipStream_t s);
// the E~ / F~ tables of the lookup-table I_l: kLutN^2 nodes {E~, F~}
hipError_t launch_lut_build(double2* table, hipStream_t s);
hipError_t launch_count(const LaunchPlan& L, unsigned long long* out, hipStream_t s);
// estimated work of the (transducer, time tile) items of one shape group (P.kperm, P.nk):
// cost[kk ntiles + t] += shells of each brick window inside tile t (cost zeroed by the caller)
hipError_t launch_tile_cost(const KParams& P, int nbricks, int tile, int ntiles, double* cost, hipStream_t s);
hipError_t launch_adjoint(const LaunchPlan& L, const void* sig, void* coef, int B, hipStream_t s);

}  // namespace patop
