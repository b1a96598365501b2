"""The multi-GPU design (sharding over transducers) exercised on one GPU with
one context per shard: the forward of the whole array is the concatenation of
the shards' forwards (no exchange), and the adjoint is the sum of the shards'
adjoints (the one all-reduce of N values per volume), each shard keeping the
whole array's sampling window t0, L.  FP64; the shards accumulate in another
order than the whole, so agreement is to rounding."""
import numpy as np
import pytest
import torch

import pat_inputs as P
from conftest import rel_l2

pytestmark = pytest.mark.gpu


def _op(p, packed, kern, mode):
    from paper_2609_29253_amd.operator import PatOperator
    h, nf = kern
    return PatOperator(packed, p.grid.n, p.grid.origin, p.grid.spacing, h, nf, p.kappa, p.sound_speed, p.fs,
                       p.t0, p.L, p.U, mode=mode, quad_n=p.quad_n, precision="fp64",
                       max_batch=p.coef.shape[0])


@pytest.mark.parametrize("mode", ["closed", "quadrature"])
@pytest.mark.parametrize("shards", [2, 3])
def test_transducer_shards_compose(gpu, shards, mode):
    from paper_2609_29253_amd.operator import build_kernel
    p = P.small_case(P.CYLINDER, n=10, K=5, L=280, B=2, seed=21)
    kern = build_kernel(p.phi_type, p.kappa, p.eir, p.sound_speed, p.fs, p.U)
    c = torch.tensor(p.coef, device=gpu)
    y = torch.tensor(p.y, device=gpu)
    whole = _op(p, p.tr.packed, kern, mode)
    s_all = whole.forward(c).cpu().numpy()
    z_all = whole.adjoint(y).cpu().numpy()
    whole.close()
    s_cat = np.zeros_like(s_all)
    z_sum = np.zeros_like(z_all)
    for r in range(shards):
        idx = np.arange(r, p.K, shards)
        op = _op(p, p.tr.packed[idx], kern, mode)
        s_cat[:, idx] = op.forward(c).cpu().numpy()
        z_sum += op.adjoint(y[:, torch.tensor(idx, device=gpu)].contiguous()).cpu().numpy()
        op.close()
    es, ez = rel_l2(s_cat, s_all), rel_l2(z_sum, z_all)
    print(f"{shards} shards, {mode}: forward {es:.2e} adjoint {ez:.2e}", flush=True)
    assert es < 1e-13 and ez < 1e-13
