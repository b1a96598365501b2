"""FP64 CPU oracle of the photoacoustic operator (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library: it is an independent plain-C transcription of the paper's
algorithms (see ``oracle.c`` for the sections, equations and algorithms each
function follows).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_l = ctypes.c_long
_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int)
_pl = ctypes.POINTER(ctypes.c_long)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.or_carlson_rf.restype = _d
        L.or_carlson_rf.argtypes = [_d, _d, _d]
        L.or_carlson_rd.restype = _d
        L.or_carlson_rd.argtypes = [_d, _d, _d]
        L.or_ellip_e.restype = _d
        L.or_ellip_e.argtypes = [_d, _d]
        L.or_ellip_f.restype = _d
        L.or_ellip_f.argtypes = [_d, _d]
        L.or_build_kernel.restype = _i
        L.or_build_kernel.argtypes = [_i, _d, _i, _pd, _pd, _l, _d, _d, _d, _i, _pd, _l, _pl, _pl]
        L.or_shell_area.restype = _d
        L.or_shell_area.argtypes = [_pd, _pd, _d, _d]
        L.or_pair_areas.restype = _l
        L.or_pair_areas.argtypes = [_pd, _pd, _d, _d, _d, _pl, _pl, _pd, _l]
        L.or_pair_areas_mode.restype = _l
        L.or_pair_areas_mode.argtypes = [_pd, _pd, _d, _d, _d, _i, _i, _pl, _pl, _pd, _l]
        L.or_quad_points.restype = None
        L.or_quad_points.argtypes = [_pd, _i, _i, _pd, _pd]
        common = [_pd, _i, _pl, _pd, _d, _pd, _l, _l, _d, _d, _d, _i, _i, _i, _i, _i, _i]
        L.or_fcoef.restype = None
        L.or_fcoef.argtypes = common + [_pd, _i, _i, _pd, _pl, _pl]
        L.or_forward.restype = None
        L.or_forward.argtypes = common + [_pd, _i, _pi, _i, _pd]
        L.or_adjoint.restype = None
        L.or_adjoint.argtypes = common + [_pd, _i, _pl, _l, _pd]
        L.or_lut_e.restype = _d
        L.or_lut_e.argtypes = [_d, _d]
        L.or_lut_entry.restype = None
        L.or_lut_entry.argtypes = [_i, _i, _pd, _pd, _pd, _pd]
        L.or_lut_set_size.restype = None
        L.or_lut_set_size.argtypes = [_i]
        L.or_num_threads.restype = _i
        L.or_set_threads.argtypes = [_i]
        _lib = L
    return _lib


def _p(a, t=_pd):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def carlson_rf(x, y, z):
    return lib().or_carlson_rf(x, y, z)


def carlson_rd(x, y, z):
    return lib().or_carlson_rd(x, y, z)


def ellip_e(phi, m):
    return lib().or_ellip_e(phi, m)


def ellip_f(phi, m):
    return lib().or_ellip_f(phi, m)


def build_kernel(phi_type, kappa, eir, c, fs, U):
    """Discrete system kernel h[n], n = n_first .. n_first + len - 1 (Eq. def_bh)."""
    cap = 1 << 20
    h = np.zeros(cap)
    nf, ln = _l(0), _l(0)
    par = _f64(eir.params())
    smp = _f64(eir.samples if eir.samples is not None else np.zeros(1))
    ns = 0 if eir.samples is None else len(eir.samples)
    rc = lib().or_build_kernel(int(phi_type), kappa, int(eir.kind), _p(par), _p(smp), ns, eir.dt,
                               c, fs, int(U), _p(h), cap, ctypes.byref(nf), ctypes.byref(ln))
    if rc != 0:
        raise RuntimeError("kernel does not fit")
    return h[: ln.value].copy(), nf.value


def kernel_of(prob):
    return build_kernel(prob.phi_type, prob.kappa, prob.eir, prob.sound_speed, prob.fs, prob.U)


def shell_area(tr_row, x, r0, r1):
    return lib().or_shell_area(_p(_f64(tr_row)), _p(_f64(x)), r0, r1)


def pair_areas(tr_row, x, c, t0, ufs):
    cap = 1 << 16
    out = np.zeros(cap)
    l0, l1 = _l(0), _l(0)
    n = lib().or_pair_areas(_p(_f64(tr_row)), _p(_f64(x)), c, t0, ufs, ctypes.byref(l0),
                            ctypes.byref(l1), _p(out), cap)
    if n < 0:
        raise RuntimeError("bin range too long")
    return l0.value, out[:n].copy()


def pair_areas_mode(tr_row, x, c, t0, ufs, mode=0, step=1):
    """Areas of one pair as a surface method uses them: exact (MODE_SURFACE),
    with the trapezoidal I_l (MODE_TRAPEZOID) or the lookup-table I_l
    (MODE_LUT), split from the coarse shells of ``step`` fine bins (Remark 1)
    when step > 1.  Returns (first bin, areas)."""
    cap = 1 << 16
    out = np.zeros(cap)
    l0, l1 = _l(0), _l(0)
    n = lib().or_pair_areas_mode(_p(_f64(tr_row)), _p(_f64(x)), c, t0, ufs, int(mode), int(step),
                                 ctypes.byref(l0), ctypes.byref(l1), _p(out), cap)
    if n < 0:
        raise RuntimeError("bin range too long")
    return l0.value, out[:n].copy()


def quad_points(tr_row, n1, n2):
    pts = np.zeros((n1 * n2, 3))
    dA = _d(0)
    lib().or_quad_points(_p(_f64(tr_row)), n1, n2, _p(pts), ctypes.byref(dA))
    return pts, dA.value


MODE_SURFACE = 0
MODE_POINT = 1
MODE_TRAPEZOID = 2
MODE_LUT = 3
LUT_SIZE = 1000


def lut_e(s, nu):
    """E(arcsin s, nu) through the lookup tables (reciprocal modulus for nu > 1)."""
    return lib().or_lut_e(float(s), float(nu))


def lut_entry(i, j):
    """Node (s_i, nu_j) of the tables (0-based) and the stored E~, F~ there."""
    v = [_d(0) for _ in range(4)]
    lib().or_lut_entry(int(i), int(j), *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v)


def lut_set_size(n):
    """Points per axis of the tables (the method uses 1000; other sizes are for
    convergence tests).  Rebuilds the tables on the next use."""
    lib().or_lut_set_size(int(n))


def _common(prob, h, nf, mode, step):
    tr = _f64(prob.tr.packed)
    n = np.ascontiguousarray(prob.grid.n, dtype=np.int64)
    org = _f64(prob.grid.origin)
    step = int(getattr(prob, "area_step", 1) if step is None else step)
    return (tr, n, org, h), (_p(tr), prob.K, _p(n, _pl), _p(org), prob.grid.spacing, _p(h), nf, len(h),
                             prob.sound_speed, prob.fs, prob.t0, prob.L, prob.U, int(mode),
                             int(prob.quad_n[0]), int(prob.quad_n[1]), step)


def fcoef(prob, k, coef=None, mode=MODE_SURFACE, kernel=None, step=None):
    """Geometric coefficients f_k (B x M) on bins Mlo..Mhi, returned with Mlo."""
    h, nf = kernel if kernel is not None else kernel_of(prob)
    h = _f64(h)
    coef = _f64(np.atleast_2d(prob.coef if coef is None else coef))
    keep, args = _common(prob, h, nf, mode, step)
    Mlo, Mhi = _l(0), _l(0)
    lib().or_fcoef(*args, _p(coef), coef.shape[0], int(k), None, ctypes.byref(Mlo), ctypes.byref(Mhi))
    f = np.zeros((coef.shape[0], Mhi.value - Mlo.value + 1))
    lib().or_fcoef(*args, _p(coef), coef.shape[0], int(k), _p(f), ctypes.byref(Mlo), ctypes.byref(Mhi))
    return f, Mlo.value


def forward(prob, coef=None, ksub=None, mode=MODE_SURFACE, kernel=None, step=None):
    """A p0 on the transducers ``ksub`` (default all): array (B, len(ksub), L)."""
    h, nf = kernel if kernel is not None else kernel_of(prob)
    h = _f64(h)
    coef = _f64(np.atleast_2d(prob.coef if coef is None else coef))
    ksub = np.arange(prob.K, dtype=np.int32) if ksub is None else np.ascontiguousarray(ksub, dtype=np.int32)
    keep, args = _common(prob, h, nf, mode, step)
    out = np.zeros((coef.shape[0], len(ksub), prob.L))
    lib().or_forward(*args, _p(coef), coef.shape[0], _p(ksub, _pi), len(ksub), _p(out))
    return out


def adjoint(prob, y=None, vsub=None, mode=MODE_SURFACE, kernel=None, step=None):
    """A^T y on the voxels ``vsub`` (default all): array (B, len(vsub))."""
    h, nf = kernel if kernel is not None else kernel_of(prob)
    h = _f64(h)
    y = _f64(prob.y if y is None else y)
    if y.ndim == 2:
        y = y[None]
    vsub = np.arange(prob.N, dtype=np.int64) if vsub is None else np.ascontiguousarray(vsub, dtype=np.int64)
    keep, args = _common(prob, h, nf, mode, step)
    out = np.zeros((y.shape[0], len(vsub)))
    lib().or_adjoint(*args, _p(y), y.shape[0], _p(vsub, _pl), len(vsub), _p(out))
    return out


def num_threads():
    return lib().or_num_threads()


def set_threads(n):
    lib().or_set_threads(int(n))
