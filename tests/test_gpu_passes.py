"""Shell windows wider than one LDS pass, on the GPU against the oracle.

At U = 24 a cylinder pair's range spans ~3700 fine bins and a planar one
~1600, so the one-wave kernels (an LDS pass of 512 shells shared by the
volumes for the cylinders, 1024 for the planar ones) walk several passes:
every pass but the first re-enters a sweep mid-quadrant (the cylinder walk then
evaluates its first edge instead of setting it), and every pass but the last
ends one before the quadrant's last edge, for one and for several volumes.
Same bar as the other parity tests: 1e-5 (FP32 I/O) and 1e-11 (FP64)
relative L2 against the FP64 oracle, and the per-row bound."""
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


def _window_bins(p):
    """Rough width in fine bins of a wave's shell window: the transducer's
    bounding diameter plus the diagonal of an 8 x 8 x 4 block of voxels."""
    dr = p.sound_speed / (p.U * p.fs)
    rads = []
    for t in p.tr.packed:
        if int(t[0]) == P.CYLINDER:
            rads.append(math.hypot(2.0 * t[12] * math.sin(0.5 * t[13]), t[14]))
        else:
            rads.append(math.hypot(t[10], t[11]))
    return (2.0 * min(rads) + math.sqrt(64 + 64 + 16) * p.grid.spacing) / dr


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("shape,B,passes", [(P.CYLINDER, 1, 512), (P.CYLINDER, 2, 256), (P.PLANAR, 4, 256)])
def test_multi_pass_windows(gpu, shape, B, passes, prec):
    from paper_2609_29253_amd.operator import PatOperator
    p = P.small_case(shape, n=6, K=2, U=24, B=B, L=260 if shape == P.CYLINDER else 200, seed=9)
    assert p.meta["window_covers_signal"]
    w = _window_bins(p)
    print(f"shape {shape} B={B} {prec}: window ~{w:.0f} fine bins, {passes} per pass", flush=True)
    assert w > 1.3 * passes
    s_ref, z_ref = O.forward(p), O.adjoint(p)
    op = PatOperator.from_problem(p, mode="closed", precision=prec)
    s = op.forward(torch.tensor(p.coef, dtype=DT[prec], device=gpu)).double().cpu().numpy()
    z = op.adjoint(torch.tensor(p.y, dtype=DT[prec], device=gpu)).double().cpu().numpy()
    op.close()
    es, ez = rel_l2(s, s_ref), rel_l2(z, z_ref)
    rs, rz = row_ratio(s, s_ref), row_ratio(z, z_ref)
    print(f"  forward {es:.3e} (worst row {rs:.3e}) adjoint {ez:.3e} (worst row {rz:.3e})", flush=True)
    assert np.linalg.norm(s_ref) > 0
    assert es < TOL[prec] and ez < TOL[prec]
    assert rs <= ROW_TAU[prec] and rz <= ROW_TAU[prec]
