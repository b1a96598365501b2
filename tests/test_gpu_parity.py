"""HIP path against the FP64 oracle, element by element, through the C ABI.

Tolerances:
  relative L2 over the whole output: FP32 variant 1e-5 (the target accuracy
  of the FP32 operator); FP64 variant 1e-11 (two independent FP64 evaluations
  of the same areas; the planar and elliptic closed forms each carry ~1e-13
  relative rounding per bin from differences of nearby edge quantities);
  per row (each transducer's signal of each volume, each volume's adjoint):
  max |gpu - oracle| <= ROW_TAU * max |oracle| over the row.
"""
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


def run_gpu(prob, mode, prec, coef=None, y=None):
    from paper_2609_29253_amd.operator import PatOperator
    coef = prob.coef if coef is None else coef
    y = prob.y if y is None else y
    B = max(coef.shape[0], y.shape[0])
    op = PatOperator.from_problem(prob, mode=mode, precision=prec, max_batch=B)
    dev = torch.device("cuda", 0)
    s = op.forward(torch.tensor(coef, dtype=DT[prec], device=dev))
    z = op.adjoint(torch.tensor(y, dtype=DT[prec], device=dev))
    torch.cuda.synchronize()
    out = s.double().cpu().numpy(), z.double().cpu().numpy()
    op.close()
    return out


def check(tag, prec, s, s_ref, z, z_ref, tol=None, tau=None):
    """Relative L2 over each output and the per-row bound."""
    tol = TOL[prec] if tol is None else tol
    tau = ROW_TAU[prec] if tau is None else tau
    es, ez = rel_l2(s, s_ref), rel_l2(z, z_ref)
    rs, rz = row_ratio(s, s_ref), row_ratio(z, z_ref)
    print(f"  {tag}: forward rel L2 {es:.3e} (worst row {rs:.3e})  adjoint rel L2 {ez:.3e} "
          f"(worst row {rz:.3e})", flush=True)
    assert np.linalg.norm(s_ref) > 0 and np.linalg.norm(z_ref) > 0
    assert es < tol and ez < tol
    assert rs <= tau and rz <= tau


SMALL = [
    # shape, U, B, n, K, L
    (P.PLANAR, 1, 1, 13, 5, 200),
    (P.PLANAR, 3, 2, 9, 4, 200),
    (P.CYLINDER, 1, 1, 13, 5, 260),
    (P.CYLINDER, 2, 3, 9, 4, 260),
    # five to eight volumes: the kernels instantiated for eight right-hand sides
    (P.PLANAR, 2, 5, 7, 3, 200),
    (P.CYLINDER, 1, 6, 7, 3, 260),
]


@pytest.mark.parametrize("mode", ["closed", "quadrature"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SMALL, ids=lambda c: f"{'pl' if c[0] == 0 else 'cy'}_U{c[1]}_B{c[2]}_n{c[3]}")
def test_small_parity(gpu, case, prec, mode):
    shape, U, B, n, K, L = case
    p = P.small_case(shape, n=n, K=K, U=U, B=B, L=L, seed=3)
    p.quad_n = (6, 5)
    omode = O.MODE_SURFACE if mode == "closed" else O.MODE_POINT
    print(f"case {p.name} U={U} B={B} {prec} {mode}", flush=True)
    s_ref = O.forward(p, mode=omode)
    z_ref = O.adjoint(p, mode=omode)
    s, z = run_gpu(p, mode, prec)
    check(p.name, prec, s, s_ref, z, z_ref)


@pytest.mark.parametrize("mode", ["closed", "quadrature"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("U,B", [(1, 1), (2, 2)])
def test_mixed_planar_and_cylinder(gpu, U, B, prec, mode):
    """An array mixing planar and cylindrical transducers (indices alternating):
    two shape groups per launch, each writing its own rows of f and W, and the
    adjoint's sum over transducers split over both groups (FP64 partial sums
    combined on the device, then cast)."""
    p = P.mixed_case(n=9, K_planar=3, K_cyl=3, U=U, B=B, L=300, seed=4)
    p.quad_n = (5, 6)
    assert list(p.tr.packed[:, 0]) == [0, 1, 0, 1, 0, 1]
    omode = O.MODE_SURFACE if mode == "closed" else O.MODE_POINT
    print(f"case {p.name} U={U} B={B} {prec} {mode}", flush=True)
    s_ref = O.forward(p, mode=omode)
    z_ref = O.adjoint(p, mode=omode)
    s, z = run_gpu(p, mode, prec)
    check(p.name, prec, s, s_ref, z, z_ref)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_point_bin_rule_on_exact_ties(gpu, prec):
    """Distances exactly on bin edges (reading 1: the upper bin), with every
    quantity of the bin rule exact in FP64 on both sides (power-of-two radial
    step, integer lattice of points and voxels).  A kernel that put a tie in
    the lower bin would move whole point contributions by one bin: ~1e-2 of a
    row, far above the per-row bound."""
    p = P.exact_tie_case()
    assert p.meta["window_covers_signal"]
    s_ref = O.forward(p, mode=O.MODE_POINT)
    z_ref = O.adjoint(p, mode=O.MODE_POINT)
    s, z = run_gpu(p, "quadrature", prec)
    check(p.name, prec, s, s_ref, z, z_ref)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_planar64_32c_full(gpu, prec):
    """Planar 64 x 32^3, every output against the oracle, plus the dot test."""
    p = P.planar64_32c()
    s_ref = O.forward(p)
    z_ref = O.adjoint(p)
    s, z = run_gpu(p, "closed", prec)
    check(p.name, prec, s, s_ref, z, z_ref)
    lhs, rhs = float(np.sum(s * p.y)), float(np.sum(z * p.coef))
    gap = abs(lhs - rhs) / (np.linalg.norm(s) * np.linalg.norm(p.y))
    print(f"planar64_32c {prec}: normalised dot gap {gap:.3e}", flush=True)
    assert gap < (1e-6 if prec == "fp32" else 1e-13)


def test_zero_input_gives_zero(gpu):
    p = P.small_case(P.CYLINDER, n=9, K=3, L=260)
    s, z = run_gpu(p, "closed", "fp32", coef=np.zeros_like(p.coef), y=np.zeros_like(p.y))
    assert not np.any(s) and not np.any(z)


def test_single_voxel_and_line_grids(gpu):
    """The smallest grids: one voxel (a brick with a single valid thread) and
    a 1 x 1 x n line, in both shapes, against the oracle."""
    for shape in (P.PLANAR, P.CYLINDER):
        for n in ((1, 1, 1), (1, 1, 6)):
            tr = P.small_case(shape, n=1, K=3, L=260, seed=6).tr
            grid = P.Grid.centred(n, 0.1e-3)
            coef = np.random.default_rng(6).random((1, grid.N))
            p = P._finish(f"line_{n[2]}", tr, grid, 40e6, 260, coef, 7)
            assert p.meta["window_covers_signal"]
            s_ref, z_ref = O.forward(p), O.adjoint(p)
            s, z = run_gpu(p, "closed", "fp64")
            check(f"{p.name} grid {n}", "fp64", s, s_ref, z, z_ref)
            assert not math.isnan(float(np.sum(s)))
