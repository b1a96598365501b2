"""The approximate surface variants on the GPU against the oracle's own
versions of them, element by element through the C ABI: the coarse area grid
of Remark 1 (each shell of `area_step` fine bins evaluated once and split
evenly), the trapezoidal cylinder I_l (Eq. trapezoid_Il) and the lookup-table
I_l (Sec. 4.2, LUT paragraph; the device builds its own tables).

Same bar as the exact method: FP32 1e-5 and FP64 1e-11 relative L2, since the
HIP path and the oracle evaluate the same approximation.  Shapes cover several
bricks and pass windows with a ragged tail; steps cover 1 < step < U, step = U
and the largest U of the tests.
"""
import numpy as np
import pytest
import torch

import oracle as O
import pat_inputs as P
from conftest import ROW_TAU, rel_l2, row_ratio

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-11}
DT = {"fp32": torch.float32, "fp64": torch.float64}
OMODE = {"closed": O.MODE_SURFACE, "trapezoid": O.MODE_TRAPEZOID, "lut": O.MODE_LUT}


def run_gpu(prob, mode, prec, step):
    from paper_2609_29253_amd.operator import PatOperator
    B = prob.coef.shape[0]
    op = PatOperator.from_problem(prob, mode=mode, precision=prec, max_batch=B, area_step=step)
    dev = torch.device("cuda", 0)
    s = op.forward(torch.tensor(prob.coef, dtype=DT[prec], device=dev))
    z = op.adjoint(torch.tensor(prob.y, dtype=DT[prec], device=dev))
    torch.cuda.synchronize()
    evals = op.query(7)
    out = s.double().cpu().numpy(), z.double().cpu().numpy(), evals
    op.close()
    return out


CASES = [
    # shape, U, step, B, n, K, L, mode
    (P.CYLINDER, 1, 1, 1, 11, 4, 260, "trapezoid"),
    (P.CYLINDER, 2, 1, 2, 9, 4, 260, "trapezoid"),
    (P.CYLINDER, 3, 3, 1, 11, 4, 260, "closed"),
    (P.CYLINDER, 4, 2, 2, 9, 3, 260, "closed"),
    (P.CYLINDER, 4, 4, 1, 9, 3, 260, "trapezoid"),
    (P.PLANAR, 3, 3, 2, 11, 4, 200, "closed"),
    (P.PLANAR, 5, 2, 1, 9, 4, 200, "closed"),
    (P.PLANAR, 2, 2, 1, 9, 3, 200, "trapezoid"),
    (P.CYLINDER, 1, 1, 1, 11, 4, 260, "lut"),
    (P.CYLINDER, 2, 1, 3, 9, 4, 260, "lut"),
    (P.CYLINDER, 4, 2, 2, 9, 3, 260, "lut"),
    (P.CYLINDER, 3, 3, 1, 11, 4, 260, "lut"),
    (P.PLANAR, 2, 1, 1, 9, 3, 200, "lut"),
]


def _id(c):
    return f"{'pl' if c[0] == 0 else 'cy'}_U{c[1]}_step{c[2]}_B{c[3]}_n{c[4]}_{c[7]}"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("case", CASES, ids=_id)
def test_variant_parity(gpu, case, prec):
    shape, U, step, B, n, K, L, mode = case
    p = P.small_case(shape, n=n, K=K, U=U, B=B, L=L, seed=5)
    p.area_step = step
    print(f"case {p.name} U={U} step={step} B={B} {mode} {prec}", flush=True)
    s_ref = O.forward(p, mode=OMODE[mode])
    z_ref = O.adjoint(p, mode=OMODE[mode])
    s, z, evals = run_gpu(p, mode, prec, step)
    es, ez = rel_l2(s, s_ref), rel_l2(z, z_ref)
    rs, rz = row_ratio(s, s_ref), row_ratio(z, z_ref)
    print(f"  forward rel L2 {es:.3e} (worst row {rs:.3e})  adjoint rel L2 {ez:.3e} (worst row {rz:.3e})  "
          f"area evaluations {evals:.0f}", flush=True)
    assert es < TOL[prec] and ez < TOL[prec]
    assert rs <= ROW_TAU[prec] and rz <= ROW_TAU[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_lut_reaches_the_nu_above_one_branch(gpu, prec):
    """Voxels on both sides of the focal line of a strongly focused element, so
    that nu = 4 R rho / (r^2 - (R - rho)^2) spans both table branches
    (nu <= 1 directly, nu > 1 by the reciprocal modulus), checked on the oracle."""
    p = P.small_case(P.CYLINDER, n=11, K=6, U=2, B=1, L=300, seed=8, spacing=0.15e-3, radius=6e-3)
    s_ref = O.forward(p, mode=O.MODE_LUT)
    z_ref = O.adjoint(p, mode=O.MODE_LUT)
    s, z, _ = run_gpu(p, "lut", prec, 1)
    es, ez = rel_l2(s, s_ref), rel_l2(z, z_ref)
    ex = rel_l2(s, O.forward(p))
    rs, rz = row_ratio(s, s_ref), row_ratio(z, z_ref)
    print(f"lut {prec}: forward {es:.3e} adjoint {ez:.3e} (worst rows {rs:.3e}, {rz:.3e}); "
          f"method error vs exact {ex:.3e}", flush=True)
    assert es < TOL[prec] and ez < TOL[prec]
    assert rs <= ROW_TAU[prec] and rz <= ROW_TAU[prec]
    assert ex < 1e-3


def test_coarse_grid_cuts_evaluations(gpu):
    """The coarse grid evaluates about 1/step as many areas (one per shell)."""
    p = P.small_case(P.CYLINDER, n=9, K=3, U=4, B=1, L=260, seed=5)
    counts = {}
    for step in (1, 2, 4):
        p.area_step = step
        counts[step] = run_gpu(p, "closed", "fp64", step)[2]
    print(f"area evaluations by step: {counts}", flush=True)
    assert counts[2] < 0.6 * counts[1] and counts[4] < 0.35 * counts[1]


def test_area_step_validation(gpu):
    from paper_2609_29253_amd import _lib
    from paper_2609_29253_amd.operator import PatOperator
    p = P.small_case(P.CYLINDER, n=5, K=2, U=2, B=1, L=260)
    with pytest.raises(_lib.PatError) as e:
        PatOperator.from_problem(p, mode="closed", area_step=3)    # > U
    assert e.value.status == 1
    with pytest.raises(_lib.PatError) as e:
        PatOperator.from_problem(p, mode="quadrature", area_step=2)
    assert e.value.status == 1
    with pytest.raises(_lib.PatError) as e:
        PatOperator.from_problem(p, mode="closed", area_step=0)
    assert e.value.status == 1
