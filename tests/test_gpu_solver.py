"""The operator inside a solver on the GPU: the autograd wrapper checked by
central differences, and projected gradient descent (monotone loss, resume
from an on-disk checkpoint).

The loss 0.5 |A c - y|^2 is quadratic in c, so central differences carry no
truncation error whatever the step: the gap to the autograd gradient
A^T (A c - y) is rounding only, and large steps keep the loss difference well
above the rounding of the loss itself.  y is white noise scaled to the RMS of
A c (an unscaled N(0, 1) would bury A c, whose physical size is ~1e-9).
FP64: |gap| <= 1e-10 max|grad| over all 1000 coordinates (eps = 1).
FP32: 1e-4 over 100 coordinates (eps = 10).
"""
import dataclasses

import numpy as np
import pytest
import torch

import pat_inputs as P

pytestmark = pytest.mark.gpu

DT = {"fp32": torch.float32, "fp64": torch.float64}


def fd_problem():
    return P.fd_cyl8_10c()


@pytest.mark.parametrize("prec,ncoord,eps,tol", [("fp64", 1000, 1.0, 1e-10), ("fp32", 100, 10.0, 1e-4)])
def test_autograd_matches_central_differences(gpu, prec, ncoord, eps, tol):
    from paper_2609_29253_amd.operator import PatOperator, apply
    p = fd_problem()
    B = 8
    op = PatOperator.from_problem(p, mode="closed", precision=prec, max_batch=B)
    dt = DT[prec]
    c = torch.tensor(p.coef[0], dtype=dt, device=gpu, requires_grad=True)
    with torch.no_grad():
        rms = float(torch.sqrt(torch.mean(op.forward(c.detach()).double() ** 2)))
    y = torch.tensor(p.y[0] * rms, dtype=dt, device=gpu)
    loss = 0.5 * torch.sum((apply(op, c) - y) ** 2)
    loss.backward()
    g = c.grad.double().cpu().numpy()
    assert np.all(np.isfinite(g)) and np.max(np.abs(g)) > 0

    idx = np.linspace(0, p.N - 1, ncoord).astype(np.int64)
    base = c.detach()
    fd = np.empty(ncoord)
    with torch.no_grad():
        for s in range(0, ncoord, B):
            ii = idx[s:s + B]
            nb = len(ii)
            plus = base.repeat(nb, 1)
            minus = base.repeat(nb, 1)
            rows = torch.arange(nb, device=gpu)
            cols = torch.as_tensor(ii, device=gpu)
            plus[rows, cols] += eps
            minus[rows, cols] -= eps
            lp = 0.5 * torch.sum((op.forward(plus) - y).double() ** 2, dim=(1, 2))
            lm = 0.5 * torch.sum((op.forward(minus) - y).double() ** 2, dim=(1, 2))
            fd[s:s + nb] = ((lp - lm) / (2 * eps)).cpu().numpy()
    gap = np.max(np.abs(fd - g[idx])) / np.max(np.abs(g))
    print(f"[fd {prec}] {ncoord} coordinates, eps {eps}: max gap / max|grad| = {gap:.3e}", flush=True)
    op.close()
    assert gap <= tol


def pgd_problem():
    full = P.pgd_cyl384_192c(n=48)
    tr = full.tr.subset(np.arange(0, full.K, 8))
    return dataclasses.replace(full, tr=tr, name="pgd_cyl48_48c")


def test_projected_gradient_monotone_and_resumable(gpu, tmp_path):
    """Monotone loss (step 0.9 / lambda_max of A^T A: the descent lemma), a
    smaller distance to the truth, a nonnegative iterate, and a resume from the
    checkpoint file written at iteration 4: the file holds that iterate bit for
    bit, the resumed run repeats the first four losses exactly and the rest to
    the forward's run-to-run rounding (its FP64 atomics sum in varying order)."""
    from paper_2609_29253_amd.operator import (PatOperator, load_checkpoint, power_iteration,
                                               projected_gradient)
    p = pgd_problem()
    op = PatOperator.from_problem(p, mode="closed", precision="fp32", max_batch=1)
    truth = torch.tensor(p.coef, dtype=torch.float32, device=gpu)
    clean = op.forward(truth)
    g = torch.Generator().manual_seed(p.meta["noise_seed"])
    noise = torch.randn(clean.shape, generator=g, dtype=torch.float64).to(gpu, torch.float32)
    y = clean + p.meta["noise_level"] * clean.abs().max() * noise
    lam = power_iteration(op, iters=10, seed=p.meta["power_seed"])
    assert lam > 0
    step = 0.9 / lam
    iters, cut = 8, 4
    snap = {}
    ck = str(tmp_path / "pgd_{it}.pt")

    def keep(it, c, losses):
        if it == cut:
            snap.update(it=it, c=c.detach().cpu().clone(), losses=list(losses))

    c_full, losses = projected_gradient(op, y, iters, step, callback=keep, checkpoint=ck, every=2)
    print(f"[pgd] lambda {lam:.4e}, losses {[f'{v:.5e}' for v in losses]}", flush=True)
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:])), "loss not monotone"
    assert losses[-1] < 0.5 * losses[0]
    err = float(torch.linalg.vector_norm(c_full - truth) / torch.linalg.vector_norm(truth))
    print(f"[pgd] |c - c_true| / |c_true| after {iters} iterations: {err:.4f}", flush=True)
    assert err < 1.0
    assert bool(torch.all(c_full >= 0))

    final = load_checkpoint(ck.replace("{it}", str(iters)))
    assert final["it"] == iters and torch.equal(final["c"], c_full.cpu()) and final["losses"] == losses
    st = load_checkpoint(ck.replace("{it}", str(cut)))
    assert st["it"] == cut and torch.equal(st["c"], snap["c"]) and st["losses"] == snap["losses"]
    c_res, losses_res = projected_gradient(op, y, iters, step, state=st)
    assert len(losses_res) == iters
    assert losses_res[:cut] == losses[:cut]
    np.testing.assert_allclose(losses_res[cut:], losses[cut:], rtol=1e-5)
    rel = float(torch.linalg.vector_norm(c_res - c_full) / torch.linalg.vector_norm(c_full))
    print(f"[pgd] resumed from the file vs uninterrupted: rel diff {rel:.3e}", flush=True)
    assert rel < 1e-5
    op.close()
