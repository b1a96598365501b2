"""pat_forward_noalloc (the forward for callers that cannot allocate) through
the C ABI against pat_forward on the same inputs: two calls in a row on one
GPU, the second with a smaller input (fewer transducers, shorter signals, one
volume), so the second reuses the static scratch that the first left filled.
Both run the same kernels, so they agree to the FP64 reordering of the
atomics in f (~1e-15 of the signal): the bar is the parity bar of the HIP
path, 1e-11 relative L2 in FP64 and 1e-5 in FP32 (FP32 I/O), with the per-row
bound.  Sizes beyond the static scratch are refused with PAT_E_UNSUPPORTED.
"""
import ctypes

import numpy as np
import pytest
import torch

import pat_inputs as P
from conftest import ROW_TAU, rel_l2, row_ratio

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-11}
DT = {"fp32": torch.float32, "fp64": torch.float64}


def both_forwards(p, prec):
    """pat_forward and pat_forward_noalloc on caller-allocated buffers."""
    from paper_2609_29253_amd import _lib
    from paper_2609_29253_amd.operator import PatOperator
    B = p.coef.shape[0]
    op = PatOperator.from_problem(p, mode="closed", precision=prec, max_batch=B)
    coef = torch.tensor(p.coef, dtype=DT[prec], device="cuda")
    ref = torch.empty((B, p.K, p.L), dtype=DT[prec], device="cuda")
    got = torch.full((B, p.K, p.L), float("nan"), dtype=DT[prec], device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = _lib.lib()
    _lib.check(L.pat_forward(op._ctx, ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(ref.data_ptr()), B,
                             stream), op._ctx)
    _lib.check(L.pat_forward_noalloc(op._ctx, ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(got.data_ptr()),
                                     B, stream), op._ctx)
    torch.cuda.synchronize()
    out = got.double().cpu().numpy(), ref.double().cpu().numpy()
    op.close()
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_forward_matches_forward_twice(gpu, prec):
    first = P.small_case(P.CYLINDER, n=12, K=5, L=300, B=2, seed=21)
    second = P.small_case(P.PLANAR, n=7, K=2, L=160, B=1, seed=22)
    for p in (first, second):
        got, ref = both_forwards(p, prec)
        e, r = rel_l2(got, ref), row_ratio(got, ref)
        print(f"{p.name} {prec}: noalloc vs forward rel L2 {e:.3e}, worst row {r:.3e}", flush=True)
        assert np.all(np.isfinite(got)) and np.linalg.norm(ref) > 0
        assert e < TOL[prec] and r <= ROW_TAU[prec]


def test_noalloc_forward_refuses_sizes_beyond_its_scratch(gpu):
    """8 transducers x 2^21 samples need 128 MiB of fine-bin scratch: refused,
    with the regular forward still available on the same context."""
    from paper_2609_29253_amd import _lib
    from paper_2609_29253_amd.operator import PatOperator
    p = P.small_case(P.PLANAR, n=4, K=8, L=1 << 21, B=1, seed=23)
    op = PatOperator.from_problem(p, mode="closed", precision="fp32")
    assert p.K * op.query(2) * 8 > 64 * (1 << 20)
    coef = torch.tensor(p.coef, dtype=torch.float32, device="cuda")
    out = torch.empty((1, p.K, p.L), dtype=torch.float32, device="cuda")
    st = _lib.lib().pat_forward_noalloc(op._ctx, ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        1, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    msg = _lib.lib().pat_last_error(op._ctx).decode()
    print(f"status {st}: {msg}", flush=True)
    assert st == 9 and "scratch" in msg
    op.close()
