"""PyTorch-facing wrapper of the patop library.

``PatOperator`` owns one library context.  ``forward``/``adjoint`` take CUDA
(HIP) tensors and launch on torch's current stream; torch provides device
memory and streams only, every step of A and A^T runs in the library's
kernels.  ``PatApply`` is the torch.autograd.Function whose backward is the
hand-written adjoint (the exact transpose of the forward, appendix on adjoint
operators).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def build_kernel(phi_type: int, kappa: float, eir, sound_speed: float, fs: float, U: int):
    """System kernel h[n] (Eq. def_bh) from the library's host builder.
    ``eir`` has fields kind, fc, sigma_t, tc, te, samples, dt (pat_inputs.Eir)."""
    e = L.Eir()
    e.kind = int(eir.kind)
    e.fc, e.sigma_t, e.t_c, e.t_e = float(eir.fc), float(eir.sigma_t), float(eir.tc), float(eir.te)
    keep = None
    if eir.samples is not None:
        keep = np.ascontiguousarray(eir.samples, dtype=np.float64)
        e.samples = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        e.n_samples = len(keep)
        e.dt = float(eir.dt)
    nf, ln = ctypes.c_int64(0), ctypes.c_int64(0)
    st = L.lib().pat_build_kernel(int(phi_type), float(kappa), ctypes.byref(e), float(sound_speed), float(fs),
                                  int(U), None, 0, ctypes.byref(nf), ctypes.byref(ln))
    h = np.zeros(ln.value)
    st = L.lib().pat_build_kernel(int(phi_type), float(kappa), ctypes.byref(e), float(sound_speed), float(fs),
                                  int(U), h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(h),
                                  ctypes.byref(nf), ctypes.byref(ln))
    L.check(st)
    del keep
    return h, nf.value


def check_geometry(packed, n, origin, spacing, kappa):
    """Host-only validation (no GPU needed); returns the distance lower bound."""
    arr = L.transducer_array(packed)
    g = L.grid_struct(n, origin, spacing)
    d = ctypes.c_double(0.0)
    st = L.lib().pat_check_geometry(arr, len(packed), ctypes.byref(g), float(kappa), ctypes.byref(d))
    L.check(st)
    return d.value


class PatOperator:
    """A and A^T for one geometry on one device."""

    def __init__(self, packed, n, origin, spacing, h, n_first, kappa, sound_speed, fs, t0, L_, U=1,
                 mode: str = "closed", quad_n: Sequence[int] = (16, 16), precision: str = "fp32",
                 max_batch: int = 1, device: int = 0, area_step: int = 1, time_tiles=None):
        self.K = len(packed)
        self.n = tuple(int(v) for v in n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.L = int(L_)
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.device = torch.device("cuda", device)
        self.max_batch = int(max_batch)
        self.mode = mode
        ctx = ctypes.c_void_p()
        L.check(L.lib().pat_create(ctypes.byref(ctx), int(device)))
        self._ctx = ctx
        arr = L.transducer_array(packed)
        g = L.grid_struct(n, origin, spacing)
        hh = np.ascontiguousarray(h, dtype=np.float64)
        kern = L.Kernel(hh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(n_first), len(hh), float(kappa))
        p = L.Params()
        p.sound_speed, p.fs, p.t0 = float(sound_speed), float(fs), float(t0)
        p.L, p.U = self.L, int(U)
        modes = {"closed": L.PAT_AREA_CLOSED, "quadrature": L.PAT_AREA_QUADRATURE,
                 "trapezoid": L.PAT_AREA_TRAPEZOID, "lut": L.PAT_AREA_LUT}
        if mode not in modes:
            raise ValueError(f"mode must be one of {sorted(modes)}")
        p.area_mode = modes[mode]
        p.area_step = int(area_step)
        p.reserved = 0
        p.quad_n1, p.quad_n2 = int(quad_n[0]), int(quad_n[1])
        p.precision = L.PAT_FP32 if precision == "fp32" else L.PAT_FP64
        p.max_batch = self.max_batch
        # time_tiles: None (cube forward), 0 (time-tile forward, automatic tile
        # width) or the tile width in area shells (a power of two, 32..512)
        if time_tiles is None:
            p.flags = 0
        else:
            t = int(time_tiles)
            if t and (t < 32 or t > 512 or t & (t - 1)):
                raise ValueError("time_tiles must be 0 or a power of two in 32..512")
            p.flags = L.PAT_FLAG_TIME_TILES | ((t.bit_length() - 1) << 8 if t else 0)
        st = L.lib().pat_set_geometry(self._ctx, arr, self.K, ctypes.byref(g), ctypes.byref(kern), ctypes.byref(p))
        L.check(st, self._ctx)

    @classmethod
    def from_problem(cls, prob, mode="closed", precision="fp32", max_batch=None, device=0, kernel=None,
                     area_step=None, time_tiles=None):
        h, nf = kernel if kernel is not None else build_kernel(prob.phi_type, prob.kappa, prob.eir,
                                                               prob.sound_speed, prob.fs, prob.U)
        B = max_batch if max_batch is not None else (prob.coef.shape[0] if prob.coef is not None else 1)
        return cls(prob.tr.packed, prob.grid.n, prob.grid.origin, prob.grid.spacing, h, nf, prob.kappa,
                   prob.sound_speed, prob.fs, prob.t0, prob.L, prob.U, mode, prob.quad_n, precision, B, device,
                   getattr(prob, "area_step", 1) if area_step is None else area_step, time_tiles)

    def query(self, what: int) -> float:
        out = ctypes.c_double(0.0)
        L.check(L.lib().pat_query(self._ctx, int(what), ctypes.byref(out)), self._ctx)
        return out.value

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _prep(self, x: torch.Tensor, inner: int):
        if x.device != self.device or x.dtype != self.dtype:
            raise ValueError(f"expected a {self.dtype} tensor on {self.device}, got {x.dtype} on {x.device}")
        x = x.contiguous()
        B = x.numel() // inner
        if B * inner != x.numel() or not 1 <= B <= self.max_batch:
            raise ValueError(f"bad shape {tuple(x.shape)} (batch must be 1..{self.max_batch})")
        return x, B

    def forward(self, coef: torch.Tensor, sparse: bool = False) -> torch.Tensor:
        """coef [B, N] (or [N]) -> signals [B, K, L].  sparse=True sums only over the
        voxels where some volume is nonzero (same result; for sparse phantoms)."""
        squeeze = coef.dim() == 1
        coef, B = self._prep(coef, self.N)
        out = torch.empty((B, self.K, self.L), dtype=self.dtype, device=self.device)
        fn = L.lib().pat_forward_sparse if sparse else L.lib().pat_forward
        st = fn(self._ctx, ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(out.data_ptr()), B, self._stream())
        L.check(st, self._ctx)
        return out[0] if squeeze else out

    def adjoint(self, sig: torch.Tensor) -> torch.Tensor:
        """signals [B, K, L] (or [K, L]) -> coef [B, N]."""
        squeeze = sig.dim() == 2
        sig, B = self._prep(sig, self.K * self.L)
        out = torch.empty((B, self.N), dtype=self.dtype, device=self.device)
        st = L.lib().pat_adjoint(self._ctx, ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(out.data_ptr()), B,
                                 self._stream())
        L.check(st, self._ctx)
        return out[0] if squeeze else out

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            torch.cuda.synchronize(self.device)
            L.lib().pat_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            if getattr(self, "_ctx", None) is not None and self._ctx.value:
                L.lib().pat_destroy(self._ctx)
        except Exception:
            pass


class PatApply(torch.autograd.Function):
    """y = A c with backward grad_c = A^T grad_y (the hand-written adjoint)."""

    @staticmethod
    def forward(ctx, coef, op: PatOperator):
        ctx.op = op
        return op.forward(coef)

    @staticmethod
    def backward(ctx, grad):
        return ctx.op.adjoint(grad), None


def apply(op: PatOperator, coef: torch.Tensor) -> torch.Tensor:
    return PatApply.apply(coef, op)


def power_iteration(op: PatOperator, iters: int = 20, seed: int = 7) -> float:
    """Largest eigenvalue of A^T A by power iteration (for a step size)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.rand(1, op.N, generator=g, dtype=torch.float64).to(op.device)
    lam = 0.0
    for _ in range(iters):
        # norms and the Rayleigh quotient in FP64: the entries of A^T A v are
        # ~1e-27 for physical units, whose squares underflow FP32
        v = v / torch.linalg.vector_norm(v)
        w = op.adjoint(op.forward(v.to(op.dtype))).double()
        lam = float(torch.sum(v * w))
        v = w
    return lam


def save_checkpoint(path: str, it: int, c: torch.Tensor, losses, step: float) -> None:
    """Projected-gradient state after iteration ``it``: the iterate (on the
    host, bit for bit), the loss history, the step size and torch's CPU random
    state, written to a temporary file and renamed over ``path`` so that a
    crash never leaves a partial checkpoint."""
    import os
    tmp = f"{path}.tmp"
    torch.save({"it": int(it), "c": c.detach().cpu().clone(), "losses": [float(v) for v in losses],
                "step": float(step), "rng_cpu": torch.get_rng_state()}, tmp)
    os.replace(tmp, path)


def load_checkpoint(path: str) -> dict:
    """A checkpoint written by ``save_checkpoint`` (tensors and plain numbers
    only: loaded with weights_only=True)."""
    st = torch.load(path, map_location="cpu", weights_only=True)
    torch.set_rng_state(st["rng_cpu"])
    return st


def projected_gradient(op: PatOperator, y: torch.Tensor, iters: int, step: float,
                       c0: Optional[torch.Tensor] = None, callback=None, state: Optional[dict] = None,
                       checkpoint: Optional[str] = None, every: int = 10):
    """c <- max(0, c - step * A^T (A c - y)); returns (c, loss history), where
    losses[j] = 0.5 |A c_j - y|^2 of the iterate entering iteration j.
    ``checkpoint``: a file written after every ``every`` iterations (and the
    last) with ``save_checkpoint``; a "{it}" in the name is replaced by the
    iteration count (one file per checkpoint), otherwise the file is rewritten.
    ``state`` (a loaded checkpoint, or a dict {'it', 'c', 'losses'}) resumes
    from that iteration with its iterate bit for bit; the operator's forward
    sums its FP64 fine-bin terms in a run-dependent order, so later iterates
    match an uninterrupted run to rounding only."""
    if state is not None:
        c = state["c"].to(op.device, op.dtype).clone()
        losses = list(state["losses"])
        start = int(state["it"])
    else:
        c = torch.zeros(1, op.N, dtype=op.dtype, device=op.device) if c0 is None else c0.clone()
        losses = []
        start = 0
    for it in range(start, iters):
        r = op.forward(c) - y
        losses.append(0.5 * float(torch.sum(r.double() ** 2)))
        c = torch.clamp(c - step * op.adjoint(r), min=0.0)
        if callback is not None:
            callback(it + 1, c, losses)
        if checkpoint is not None and ((it + 1) % every == 0 or it + 1 == iters):
            save_checkpoint(checkpoint.replace("{it}", str(it + 1)), it + 1, c, losses, step)
    return c, losses
