"""ctypes binding of the patop C ABI (include/patop.h).

Argument marshalling only: every step of the operator runs in the HIP library.
Loading fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpatop.so")

PAT_OK = 0
STATUS_NAMES = ["PAT_OK", "PAT_E_ARG", "PAT_E_FRAME", "PAT_E_SHAPE", "PAT_E_SEPARATION", "PAT_E_KERNEL",
                "PAT_E_STATE", "PAT_E_DEVICE", "PAT_E_OOM", "PAT_E_UNSUPPORTED"]

PAT_PLANAR, PAT_CYLINDER = 0, 1
PAT_AREA_CLOSED, PAT_AREA_QUADRATURE, PAT_AREA_TRAPEZOID, PAT_AREA_LUT = 0, 1, 2, 3
ABI_VERSION = 4
PAT_FP32, PAT_FP64 = 0, 1
PAT_PHI_CONE, PAT_PHI_WENDLAND2 = 0, 1
PAT_EIR_GAUSS_COS, PAT_EIR_SAMPLED = 0, 1
PAT_FLAG_TIME_TILES = 1

EXPORTED = ["pat_create", "pat_set_geometry", "pat_forward", "pat_forward_sparse", "pat_forward_noalloc",
            "pat_adjoint",
            "pat_build_kernel", "pat_check_geometry", "pat_query", "pat_probe_peak", "pat_status_string",
            "pat_last_error", "pat_destroy"]


class PatError(RuntimeError):
    def __init__(self, status, msg=""):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}" if msg else name)
        self.status = status


class Transducer(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("c0", ctypes.c_double * 3), ("e1", ctypes.c_double * 3), ("e2", ctypes.c_double * 3),
                ("half_w", ctypes.c_double), ("half_h", ctypes.c_double),
                ("radius", ctypes.c_double), ("theta_max", ctypes.c_double), ("half_len", ctypes.c_double),
                ("unused", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64 * 3), ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double)]


class Kernel(ctypes.Structure):
    _fields_ = [("h", ctypes.POINTER(ctypes.c_double)), ("n_first", ctypes.c_int64), ("len", ctypes.c_int64),
                ("kappa", ctypes.c_double)]


class Eir(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("fc", ctypes.c_double), ("sigma_t", ctypes.c_double), ("t_c", ctypes.c_double),
                ("t_e", ctypes.c_double), ("samples", ctypes.POINTER(ctypes.c_double)),
                ("n_samples", ctypes.c_int64), ("dt", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("sound_speed", ctypes.c_double), ("fs", ctypes.c_double), ("t0", ctypes.c_double),
                ("L", ctypes.c_int32), ("U", ctypes.c_int32), ("area_mode", ctypes.c_int32),
                ("quad_n1", ctypes.c_int32), ("quad_n2", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("flags", ctypes.c_int32), ("area_step", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2609_29253_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback implementation")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    c = ctypes
    L.pat_create.argtypes = [P(c.c_void_p), c.c_int32]
    L.pat_set_geometry.argtypes = [c.c_void_p, P(Transducer), c.c_int32, P(Grid), P(Kernel), P(Params)]
    L.pat_forward.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p, c.c_int32, c.c_void_p]
    L.pat_forward_sparse.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p, c.c_int32, c.c_void_p]
    L.pat_forward_noalloc.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p, c.c_int32, c.c_void_p]
    L.pat_adjoint.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p, c.c_int32, c.c_void_p]
    L.pat_build_kernel.argtypes = [c.c_int32, c.c_double, P(Eir), c.c_double, c.c_double, c.c_int32,
                                   P(c.c_double), c.c_int64, P(c.c_int64), P(c.c_int64)]
    L.pat_check_geometry.argtypes = [P(Transducer), c.c_int32, P(Grid), c.c_double, P(c.c_double)]
    L.pat_query.argtypes = [c.c_void_p, c.c_int32, P(c.c_double)]
    L.pat_probe_peak.argtypes = [c.c_int32, P(c.c_double)]
    L.pat_status_string.argtypes = [c.c_int32]
    L.pat_status_string.restype = c.c_char_p
    L.pat_last_error.argtypes = [c.c_void_p]
    L.pat_last_error.restype = c.c_char_p
    L.pat_destroy.argtypes = [c.c_void_p]
    L.pat_destroy.restype = None
    for name in ("pat_create", "pat_set_geometry", "pat_forward", "pat_forward_sparse", "pat_forward_noalloc",
                 "pat_adjoint",
                 "pat_build_kernel", "pat_check_geometry", "pat_query", "pat_probe_peak"):
        getattr(L, name).restype = c.c_int32
    _lib = L
    return L


def check(status, ctx=None):
    if status != PAT_OK:
        msg = ""
        if ctx is not None:
            raw = lib().pat_last_error(ctx)
            msg = raw.decode() if raw else ""
        raise PatError(status, msg)


def transducer_array(packed):
    """(K, 16) packed float64 rows (shape, c0, e1, e2, half_w, half_h, radius,
    theta_max, half_len, unused) -> ctypes array of Transducer."""
    K = len(packed)
    arr = (Transducer * K)()
    for k, row in enumerate(packed):
        t = arr[k]
        t.shape = int(row[0])
        for a in range(3):
            t.c0[a], t.e1[a], t.e2[a] = float(row[1 + a]), float(row[4 + a]), float(row[7 + a])
        t.half_w, t.half_h = float(row[10]), float(row[11])
        t.radius, t.theta_max, t.half_len = float(row[12]), float(row[13]), float(row[14])
    return arr


def grid_struct(n, origin, spacing):
    g = Grid()
    for a in range(3):
        g.n[a] = int(n[a])
        g.origin[a] = float(origin[a])
    g.spacing = float(spacing)
    return g


def probe_peak(device: int = 0) -> dict:
    """Measured FP64 / FP32 FMA throughput of the device (pat_probe_peak)."""
    out = (ctypes.c_double * 4)()
    check(lib().pat_probe_peak(int(device), out))
    return {"fp64_flops": out[0], "fp32_flops": out[1], "compute_units": int(out[2]), "clock_ghz": out[3]}
