"""Failure handling of the C ABI on a real context, forced from the host.

Every refused call is refused by a host-side check before anything is
launched: a context without a geometry (PAT_E_STATE), a system kernel with a
non-finite tap or no taps (PAT_E_KERNEL, after which the context has dropped its
previous geometry), NULL or misaligned buffers and batches out of range
(PAT_E_ARG), invalid parameters (PAT_E_ARG), and the window-truncation flag of
pat_query(4) for a recording too short for the farthest arrivals.  After the
refused calls the context still computes what a fresh one computes.
"""
import ctypes

import numpy as np
import pytest
import torch

import pat_inputs as P

pytestmark = pytest.mark.gpu

OK, E_ARG, E_KERNEL, E_STATE = 0, 1, 5, 6


def ptr(t, offset=0):
    return ctypes.c_void_p(t.data_ptr() + offset)


class Ctx:
    """One library context built through the C ABI (not the torch wrapper)."""

    def __init__(self):
        from paper_2609_29253_amd import _lib
        self.L = _lib.lib()
        self.lib = _lib
        self.h = ctypes.c_void_p()
        assert self.L.pat_create(ctypes.byref(self.h), 0) == OK

    def set_geometry(self, p, h=None, n_first=None, precision=0, max_batch=1, L=None, flags=0):
        from paper_2609_29253_amd.operator import build_kernel
        if h is None:
            h, n_first = build_kernel(p.phi_type, p.kappa, p.eir, p.sound_speed, p.fs, p.U)
        hh = np.ascontiguousarray(h, dtype=np.float64)
        kern = self.lib.Kernel(hh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(n_first), len(hh),
                               float(p.kappa))
        prm = self.lib.Params()
        prm.sound_speed, prm.fs, prm.t0 = p.sound_speed, p.fs, p.t0
        prm.L, prm.U = int(p.L if L is None else L), int(p.U)
        prm.area_mode, prm.quad_n1, prm.quad_n2 = self.lib.PAT_AREA_CLOSED, 4, 4
        prm.precision, prm.max_batch, prm.flags = precision, max_batch, flags
        prm.area_step, prm.reserved = 1, 0
        arr = self.lib.transducer_array(p.tr.packed)
        g = self.lib.grid_struct(p.grid.n, p.grid.origin, p.grid.spacing)
        return self.L.pat_set_geometry(self.h, arr, len(p.tr.packed), ctypes.byref(g), ctypes.byref(kern),
                                       ctypes.byref(prm))

    def query(self, what):
        out = ctypes.c_double(-1.0)
        st = self.L.pat_query(self.h, what, ctypes.byref(out))
        return st, out.value

    def message(self):
        return (self.L.pat_last_error(self.h) or b"").decode()

    def close(self):
        torch.cuda.synchronize()
        self.L.pat_destroy(self.h)


def test_state_before_geometry_and_after_a_failed_one(gpu):
    p = P.small_case(P.CYLINDER, n=6, K=3, L=200, seed=1)
    c = Ctx()
    coef = torch.zeros(p.N, device="cuda")
    sig = torch.zeros(p.K * p.L, device="cuda")
    for fn in ("pat_forward", "pat_forward_sparse", "pat_forward_noalloc"):
        assert getattr(c.L, fn)(c.h, ptr(coef), ptr(sig), 1, None) == E_STATE
    assert c.L.pat_adjoint(c.h, ptr(sig), ptr(coef), 1, None) == E_STATE
    assert c.query(0)[0] == E_STATE
    assert "set_geometry" in c.message()
    # a geometry that succeeds, then one whose kernel is refused: the context
    # drops the first and refuses to run until a geometry succeeds again
    assert c.set_geometry(p) == OK
    assert c.L.pat_forward(c.h, ptr(coef), ptr(sig), 1, None) == OK
    bad = np.array([0.0, 1.0, np.nan, 0.5])
    assert c.set_geometry(p, h=bad, n_first=0) == E_KERNEL
    assert "kernel" in c.message()
    assert c.L.pat_forward(c.h, ptr(coef), ptr(sig), 1, None) == E_STATE
    assert c.set_geometry(p, h=np.zeros(0), n_first=0) == E_KERNEL
    assert c.set_geometry(p) == OK
    assert c.L.pat_forward(c.h, ptr(coef), ptr(sig), 1, None) == OK
    c.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_argument_errors_launch_nothing_and_leave_the_context_usable(gpu, prec):
    from paper_2609_29253_amd.operator import PatOperator
    p = P.small_case(P.PLANAR, n=7, K=3, L=200, seed=2, B=2)
    dt = torch.float64 if prec else torch.float32
    es = 8 if prec else 4
    c = Ctx()
    assert c.set_geometry(p, precision=prec, max_batch=2) == OK
    coef = torch.tensor(p.coef, dtype=dt, device="cuda")
    sig = torch.zeros((2, p.K, p.L), dtype=dt, device="cuda")
    for fn in ("pat_forward", "pat_forward_sparse", "pat_forward_noalloc"):
        f = getattr(c.L, fn)
        assert f(c.h, ptr(coef), ptr(sig), 0, None) == E_ARG
        assert f(c.h, ptr(coef), ptr(sig), 3, None) == E_ARG
        assert f(c.h, None, ptr(sig), 1, None) == E_ARG
        assert f(c.h, ptr(coef), None, 1, None) == E_ARG
        assert f(c.h, ptr(coef, es // 2), ptr(sig), 1, None) == E_ARG
        assert f(c.h, ptr(coef), ptr(sig, es // 2), 1, None) == E_ARG
        assert "aligned" in c.message()
    assert c.L.pat_adjoint(c.h, ptr(sig, 2), ptr(coef), 1, None) == E_ARG
    assert c.L.pat_adjoint(c.h, ptr(sig), ptr(coef), 3, None) == E_ARG
    assert c.query(99)[0] == E_ARG
    # the context is intact: its forward equals a fresh operator's
    assert c.L.pat_forward(c.h, ptr(coef), ptr(sig), 2, None) == OK
    torch.cuda.synchronize()
    op = PatOperator.from_problem(p, mode="closed", precision="fp64" if prec else "fp32", max_batch=2)
    ref = op.forward(coef)
    torch.cuda.synchronize()
    d = float(torch.max(torch.abs(sig.double() - ref.double())) / torch.max(torch.abs(ref.double())))
    print(f"precision {prec}: context after refused calls vs a fresh operator: {d:.3e}", flush=True)
    assert d < (1e-6 if prec == 0 else 1e-13)
    op.close()
    c.close()


def test_invalid_parameters_are_refused(gpu):
    p = P.small_case(P.CYLINDER, n=6, K=3, L=200, seed=3)
    c = Ctx()
    assert c.set_geometry(p, precision=7) == E_ARG
    assert c.set_geometry(p, max_batch=0) == E_ARG
    assert c.set_geometry(p, flags=4) == E_ARG            # an unknown flag bit
    assert c.set_geometry(p, flags=5 << 8) == E_ARG       # a tile width without the tile forward
    assert c.set_geometry(p, flags=1 | (3 << 8)) == E_ARG  # a tile width below 32 shells
    assert c.set_geometry(p, flags=1 | (6 << 8)) == OK
    assert c.query(9) == (OK, 64.0)
    assert c.set_geometry(p) == OK
    assert c.query(9) == (OK, 0.0)
    c.close()


def test_truncation_flag(gpu):
    """pat_query(4) is 1 when an arrival can fall after the last sample (the
    recording is shorter than the farthest voxel-to-surface distance plus the
    kernel's length) and 0 when it cannot."""
    p = P.small_case(P.CYLINDER, n=6, K=3, L=260, seed=4)
    c = Ctx()
    assert c.set_geometry(p, L=1000) == OK
    full = c.query(4)
    assert c.set_geometry(p, L=40) == OK
    short = c.query(4)
    print(f"truncation flag: L = 1000 -> {full[1]}, L = 40 -> {short[1]}", flush=True)
    assert full == (OK, 0.0) and short == (OK, 1.0)
    c.close()
