"""Degenerate geometries on the GPU against the oracle: voxels on a cylinder's
focal line (rho = 0, where Phi is always clamped and nu = 0), voxels in the
plane of a cylinder's axial ends and of a planar rectangle's edges (folded
intervals that touch 0 or vanish), voxels on a planar transducer's axis, and
patches smaller than a fine bin (whole quadrants inside one or two bins).
The areas are continuous across these boundaries, so the two sides agree to
rounding even where they round a coordinate to opposite sides of a fold."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import pat_inputs as P
from conftest import ROW_TAU, rel_l2, row_ratio

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-11}
DT = {"fp32": torch.float32, "fp64": torch.float64}


def _problem(rows, name, L=320):
    tr = P.Transducers(np.array(rows))
    grid = P.Grid.centred(11, 0.1e-3)
    coef = np.random.default_rng(3).random((1, grid.N))
    return P._finish(name, tr, grid, 40e6, L, coef, 4)


def _cases():
    """Radii and the plane distance carry the irrational factor of the small
    cases, so that no voxel-to-surface corner distance lands exactly on a bin
    edge (there the end point of a level curve switches between clamped and
    interior with an infinite derivative, and the two sides' roundings decide
    it differently); the degenerate positions themselves (focal line, axial end
    planes, rectangle edges) stay on voxel planes."""
    z = [0.0, 0.0, 1.0]
    g = 1.0 + math.sqrt(2.0) * 1e-3
    return {
        # focal line along z through the grid centre: the voxels (0, 0, z) have rho = 0;
        # the axial ends at z = +-0.3 mm pass through voxel planes
        "cyl_focal_line": _problem([P.cylinder([0, 0, 0], z, [1, 0, 0], 4e-3 * g, 0.4, 0.3e-3),
                                    P.cylinder([0, 0, 0], z, [0, 1, 0], 3.5e-3 * g, 0.6, 0.2e-3)], "cyl_rho0"),
        # focal line along x through the grid: rho = 0 on a row of voxels, axial ends inside the grid
        "cyl_axis_x": _problem([P.cylinder([0, 0, 0], [1, 0, 0], [0, 0, 1], 5e-3 * g, 0.3, 0.2e-3)], "cyl_x"),
        # planar rectangles facing the grid whose edges lie on voxel planes, centred on the z axis
        "planar_edges": _problem([P.planar([0, 0, 3e-3 * g], [1, 0, 0], [0, 1, 0], 0.3e-3, 0.2e-3),
                                  P.planar([0, 0, -3e-3 * g], [0, 1, 0], [1, 0, 0], 0.5e-3, 0.1e-3)], "pl_edges"),
        # patches of a few tens of micrometres (a bin is 37.5 um): most quadrants lie
        # inside one or two bins, so a cylinder walk's set first edge (below the nearest
        # corner) and set last edge (past the farthest) bound a single evaluated edge or
        # none, and a planar walk crosses all its corners in one bin.  The areas are
        # differences of squared distances ~(D / a)^2 ~ 1e4 times larger than
        # themselves (D = 3-4 mm, a = 25-35 um), which FP64 still resolves to ~1e-12
        "tiny_patches": _problem([P.cylinder([0, 0, 0], z, [1, 0, 0], 4e-3 * g, 8e-3, 25e-6),
                                  P.cylinder([0, 0, 0.2e-3], [1, 0, 0], [0, 1, 0], 3e-3 * g, 1e-2, 30e-6),
                                  P.planar([0, 0, 3e-3 * g], [1, 0, 0], [0, 1, 0], 35e-6, 25e-6)], "tiny"),
    }


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("mode", ["closed", "lut"])
@pytest.mark.parametrize("case", ["cyl_focal_line", "cyl_axis_x", "planar_edges", "tiny_patches"])
def test_degenerate_geometry(gpu, case, mode, prec):
    from paper_2609_29253_amd.operator import PatOperator
    p = _cases()[case]
    assert p.meta["window_covers_signal"]
    omode = O.MODE_SURFACE if mode == "closed" else O.MODE_LUT
    s_ref, z_ref = O.forward(p, mode=omode), O.adjoint(p, mode=omode)
    op = PatOperator.from_problem(p, mode=mode, precision=prec)
    s = op.forward(torch.tensor(p.coef, dtype=DT[prec], device=gpu)).double().cpu().numpy()
    z = op.adjoint(torch.tensor(p.y, dtype=DT[prec], device=gpu)).double().cpu().numpy()
    op.close()
    es, ez = rel_l2(s, s_ref), rel_l2(z, z_ref)
    rs, rz = row_ratio(s, s_ref), row_ratio(z, z_ref)
    print(f"{case} {mode} {prec}: forward {es:.3e} (worst row {rs:.3e}) adjoint {ez:.3e} (worst row {rz:.3e})",
          flush=True)
    assert np.all(np.isfinite(s)) and np.all(np.isfinite(z))
    assert np.linalg.norm(s_ref) > 0
    assert es < TOL[prec] and ez < TOL[prec]
    assert rs <= ROW_TAU[prec] and rz <= ROW_TAU[prec]


def test_size_limits_are_rejected(gpu):
    """Sizes beyond the library's limits fail with PAT_E_UNSUPPORTED, before
    any product of them can overflow: 2^31 voxels or more (also with extents
    whose product exceeds 2^63) and U above 65536.  The grid keeps its spacing
    small enough to stay clear of the transducers."""
    from paper_2609_29253_amd import _lib
    from paper_2609_29253_amd.operator import PatOperator, build_kernel
    p = P.small_case(P.PLANAR, n=5, K=2, U=1, B=1, L=64)
    h, nf = build_kernel(p.phi_type, p.kappa, p.eir, p.sound_speed, p.fs, p.U)
    args = (p.tr.packed, p.grid.origin, h, nf, p.kappa, p.sound_speed, p.fs, p.t0, p.L)

    def make(n, spacing, U=1):
        packed, origin, hh, nff, kappa, c, fs, t0, L_ = args
        return PatOperator(packed, n, origin, spacing, hh, nff, kappa, c, fs, t0, L_, U)

    for n in [(2048, 1024, 1024), (1 << 40, 1 << 40, 1 << 40)]:
        with pytest.raises(_lib.PatError) as e:
            make(n, 1e-15)
        assert e.value.status == 9, n
    with pytest.raises(_lib.PatError) as e:
        make(p.grid.n, p.grid.spacing, U=70000)
    assert e.value.status == 9
    make(p.grid.n, p.grid.spacing).close()      # the same system within the limits is accepted
