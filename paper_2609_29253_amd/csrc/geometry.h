// Host-only geometry helpers of the patop library (no HIP): transducer
// bounding spheres, the grid's box and the validation behind
// pat_check_geometry.  Plain C++, so that it also builds and runs under the
// CPU sanitizers.  Not part of the ABI.
#pragma once

#include "patop.h"

namespace patop {
namespace geom {

double dot3(const double* a, const double* b);
void cross3(const double* a, const double* b, double* o);
// centre and radius of a sphere containing the transducer surface (Sec. 4.1
// rectangle, Sec. 4.2 cylinder patch)
void bounding_sphere(const pat_transducer& t, double cen[3], double& rad);
// box of the voxel centres
void grid_box(const pat_grid& g, double lo[3], double hi[3]);

}  // namespace geom
}  // namespace patop
