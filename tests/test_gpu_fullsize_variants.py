"""The approximate surface variants at full size, in the launch configuration
bench.py --next times, against the oracle's own version of each variant on
sampled outputs: the 128^3 x 256-cylinder workload with the trapezoidal and
the lookup-table I_l, and its U = 4 version with the coarse area grid
(area_step 2 and 4).  FP32 I/O, bar 1e-5 relative L2 per sampled set, as for
the exact method."""
import numpy as np
import pytest
import torch

import oracle as O
import pat_inputs as P
from conftest import ROW_TAU_FULL, rel_l2, row_ratio

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

KS = {1: np.array([0, 131], dtype=np.int32), 4: np.array([77], dtype=np.int32)}
_cache = {}


def _problem(U):
    if U not in _cache:
        _cache[U] = P.cyl256_128c() if U == 1 else P.cyl256_128c(U=U)
    return _cache[U]


@pytest.mark.parametrize("mode,U,step", [("trapezoid", 1, 1), ("lut", 1, 1), ("closed", 4, 2), ("closed", 4, 4)])
def test_variant_at_full_size(gpu, mode, U, step):
    from paper_2609_29253_amd.operator import PatOperator
    p = _problem(U)
    vs = np.linspace(0, p.N - 1, 384).astype(np.int64)
    ks = KS[U]
    omode = {"closed": O.MODE_SURFACE, "trapezoid": O.MODE_TRAPEZOID, "lut": O.MODE_LUT}[mode]
    print(f"{p.name} {mode} U={U} step={step}: oracle on transducers {ks.tolist()} and {len(vs)} voxels", flush=True)
    s_ref = O.forward(p, ksub=ks, mode=omode, step=step)
    z_ref = O.adjoint(p, vsub=vs, mode=omode, step=step)
    op = PatOperator.from_problem(p, mode=mode, precision="fp32", area_step=step)
    s = op.forward(torch.tensor(p.coef, dtype=torch.float32, device=gpu))
    z = op.adjoint(torch.tensor(p.y, dtype=torch.float32, device=gpu))
    s = s[:, torch.tensor(ks, device=gpu).long()].double().cpu().numpy()
    z = z[:, torch.tensor(vs, device=gpu)].double().cpu().numpy()
    op.close()
    es, ez = rel_l2(s, s_ref), rel_l2(z, z_ref)
    rs, rz = row_ratio(s, s_ref), row_ratio(z, z_ref)
    print(f"  forward {es:.3e} (worst row {rs:.3e})  adjoint {ez:.3e} (worst row {rz:.3e})", flush=True)
    assert es < 1e-5 and ez < 1e-5
    assert rs <= ROW_TAU_FULL["fp32"] and rz <= ROW_TAU_FULL["fp32"]
