"""Run-to-run determinism of the HIP path.

The forward adds each work-group's FP64 LDS window into f with FP64 atomics,
whose order varies from run to run, so f differs between runs by a few FP64
ulps; the FP64 temporal stage then rounds to the output type.  Two forwards of
the same input may therefore differ by at most one unit in the last place of
the FP32 output, except near a zero crossing of the signal, where the FP64
reordering difference itself (~1e-14 of the row's largest sample: FP64
rounding times the zero-mean kernel's cancellation) exceeds the FP32 ulp of
the tiny sample; in FP64 the samples differ by ~1e-13 of the row's largest.  The adjoint sums over transducers in a fixed
order per voxel when one work-group owns all of a voxel's transducers (the
benchmark's workload: 8192 bricks fill the device with one transducer chunk):
it is then bitwise reproducible.  When the transducers are split over several
work-groups (small grids, which have few bricks) or over two shape groups, it
combines FP64 partial sums with atomics and is held to the same bar as the
forward.
"""
import numpy as np
import pytest
import torch

import pat_inputs as P
from conftest import fp32_repeat_ok, ulp_distance32

pytestmark = pytest.mark.gpu

DT = {"fp32": torch.float32, "fp64": torch.float64}


def twice(p, prec, mode="closed", runs=3):
    from paper_2609_29253_amd.operator import PatOperator
    op = PatOperator.from_problem(p, mode=mode, precision=prec, max_batch=p.coef.shape[0])
    c = torch.tensor(p.coef, dtype=DT[prec], device="cuda")
    y = torch.tensor(p.y, dtype=DT[prec], device="cuda")
    outs = [(op.forward(c).cpu().numpy(), op.adjoint(y).cpu().numpy()) for _ in range(runs)]
    op.close()
    return outs


@pytest.mark.parametrize("mode", ["closed", "quadrature"])
@pytest.mark.parametrize("name", ["small_cylinder", "small_planar", "mixed"])
def test_repeat_runs_fp32(gpu, name, mode):
    if name == "mixed":
        p = P.mixed_case(n=13, K_planar=3, K_cyl=3, L=300, seed=2, B=2)
    else:
        p = P.small_case(P.CYLINDER if name == "small_cylinder" else P.PLANAR, n=16, K=5,
                         L=260 if name == "small_cylinder" else 200, seed=2, B=2)
    p.quad_n = (8, 8)
    outs = twice(p, "fp32", mode)
    s0, z0 = outs[0]
    for s, z in outs[1:]:
        ds, dz = fp32_repeat_ok(s0, s), fp32_repeat_ok(z0, z)
        print(f"{p.name} {mode}: forward {ds} ulp, adjoint {dz} ulp (raw {ulp_distance32(s0, s)} / "
              f"{ulp_distance32(z0, z)}), {int(np.sum(s0 != s))} / {s.size} samples differ", flush=True)
        assert ds <= 1 and dz <= 1


def test_repeat_runs_fp64(gpu):
    p = P.small_case(P.CYLINDER, n=16, K=5, L=260, seed=2, B=1)
    outs = twice(p, "fp64")
    s0, z0 = outs[0]
    for s, z in outs[1:]:
        d = float(np.max(np.abs(s - s0)) / np.max(np.abs(s0)))
        e = float(np.max(np.abs(z - z0)) / np.max(np.abs(z0)))
        print(f"{p.name} fp64: forward / adjoint max difference {d:.3e} / {e:.3e} of the largest", flush=True)
        assert d < 1e-13 and e < 1e-14


@pytest.mark.slow
def test_repeat_runs_headline_workload(gpu):
    """The benchmark's workload (128^3 voxels, 256 cylinders), FP32 I/O."""
    p = P.cyl256_128c()
    outs = twice(p, "fp32", runs=2)
    (s0, z0), (s1, z1) = outs
    ds = fp32_repeat_ok(s0, s1)
    print(f"cyl256_128c: forward {ds} ulp between runs ({int(np.sum(s0 != s1))} of {s0.size} samples differ), "
          f"adjoint bitwise equal {np.array_equal(z0, z1)}", flush=True)
    assert ds <= 1 and np.array_equal(z0, z1)
