"""Seeded synthetic inputs for the matrix-free photoacoustic operator.

This module only builds *inputs*: transducer poses, voxel grids, coefficient
phantoms, electrical-impulse-response (EIR) parameters, sampling parameters
and random right-hand sides.  It contains none of the operator's arithmetic
(no shell areas, no system kernel, no convolution), so that both the FP64
oracle and the HIP path can consume exactly the same inputs without sharing
any code that computes the method.

All quantities are SI (metres, seconds, hertz, metres per second).

Geometry conventions (paper: planar frame in Sec. 4.1, Eq. plane_param;
cylinder frame in Sec. 4.2, Eq. cylinder_param):

* planar transducer: centre ``c0``, orthonormal ``e1`` (half-size
  ``half_w`` along it, the paper's L1) and ``e2`` (half-size ``half_h``, L2);
  the normal ``e1 x e2`` faces the sample.
* cylindrical transducer: ``c0`` is the centre of the focal line, ``e1`` the
  cylinder axis (half-length ``half_len``, the paper's L_z), the surface point
  at angle 0 is ``c0 + radius*e2``; angular half-aperture ``theta_max``.

A transducer is packed as 16 doubles (see ``TR_FIELDS``); the C-ABI struct and
the oracle read the same order.
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import List, Optional, Sequence

import numpy as np

PLANAR = 0
CYLINDER = 1

PHI_CONE = 0        # phi(r) = max(0, 1 - r/kappa)            (Sec. 5.1)
PHI_WENDLAND2 = 1   # phi(r) = max(0, 1 - r/kappa)^2          (Sec. 2.7)

EIR_GAUSS_COS = 0   # e(t) = cos(2 pi fc (t - tc)) exp(-(t - tc)^2 / (2 sigma^2)) on [0, Te]
EIR_SAMPLED = 1     # piecewise-linear interpolant of samples e(j*dt), j = 0..n-1

# packed transducer layout: shape, c0[3], e1[3], e2[3], half_w, half_h, radius,
# theta_max, half_len, pad
TR_FIELDS = 16

SOUND_SPEED = 1500.0


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


@dataclasses.dataclass
class Transducers:
    """K transducers, packed as a (K, 16) float64 array."""
    packed: np.ndarray

    @property
    def K(self) -> int:
        return int(self.packed.shape[0])

    def subset(self, idx: Sequence[int]) -> "Transducers":
        return Transducers(np.ascontiguousarray(self.packed[np.asarray(idx)]))


def planar(c0, e1, e2, half_w, half_h) -> np.ndarray:
    row = np.zeros(TR_FIELDS)
    row[0] = PLANAR
    row[1:4], row[4:7], row[7:10] = c0, e1, e2
    row[10], row[11] = half_w, half_h
    return row


def cylinder(c0, e1, e2, radius, theta_max, half_len) -> np.ndarray:
    row = np.zeros(TR_FIELDS)
    row[0] = CYLINDER
    row[1:4], row[4:7], row[7:10] = c0, e1, e2
    row[12], row[13], row[14] = radius, theta_max, half_len
    return row


@dataclasses.dataclass
class Grid:
    """Uniform voxel-centre grid: x = origin + (ix, iy, iz) * spacing,
    flattened index i = ix + n[0] * (iy + n[1] * iz)."""
    n: tuple
    origin: tuple
    spacing: float

    @property
    def N(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @staticmethod
    def centred(n, spacing) -> "Grid":
        n = tuple(int(v) for v in (n if np.ndim(n) else (n, n, n)))
        origin = tuple(-(v - 1) / 2.0 * spacing for v in n)
        return Grid(n, origin, float(spacing))

    def coords(self) -> np.ndarray:
        """(N, 3) voxel centres in flattened order (x fastest)."""
        ix = np.arange(self.n[0]) * self.spacing + self.origin[0]
        iy = np.arange(self.n[1]) * self.spacing + self.origin[1]
        iz = np.arange(self.n[2]) * self.spacing + self.origin[2]
        Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def half_diagonal(self) -> float:
        return 0.5 * self.spacing * math.sqrt(sum((v - 1) ** 2 for v in self.n))


@dataclasses.dataclass
class Eir:
    kind: int = EIR_GAUSS_COS
    fc: float = 5e6
    sigma_t: float = 0.0
    tc: float = 0.0
    te: float = 0.0
    samples: Optional[np.ndarray] = None
    dt: float = 0.0

    @staticmethod
    def gauss_cos(fc=5e6, frac_bw=0.6, n_sigma=5.0) -> "Eir":
        """Gaussian-windowed cosine; ``frac_bw`` is the -6 dB (half-amplitude)
        fractional bandwidth, truncated at +-n_sigma standard deviations and
        shifted so the support is [0, Te] (causal, as the EIR assumption asks)."""
        sigma_f = frac_bw * fc / 2.0 / math.sqrt(2.0 * math.log(2.0))
        sigma_t = 1.0 / (2.0 * math.pi * sigma_f)
        return Eir(EIR_GAUSS_COS, fc, sigma_t, n_sigma * sigma_t, 2 * n_sigma * sigma_t)

    def params(self) -> np.ndarray:
        return np.array([self.fc, self.sigma_t, self.tc, self.te], dtype=np.float64)


@dataclasses.dataclass
class Problem:
    """Everything that defines one operator instance, plus its inputs."""
    name: str
    tr: Transducers
    grid: Grid
    phi_type: int
    kappa: float
    eir: Eir
    sound_speed: float
    fs: float
    L: int
    U: int
    t0: float
    quad_n: tuple = (16, 16)
    coef: Optional[np.ndarray] = None       # (B, N) float64
    y: Optional[np.ndarray] = None          # (B, K, L) float64
    meta: dict = dataclasses.field(default_factory=dict)
    area_step: int = 1                      # coarse area grid: fine bins per evaluated shell

    @property
    def K(self):
        return self.tr.K

    @property
    def N(self):
        return self.grid.N

    def describe(self) -> dict:
        d = dict(name=self.name, N=self.N, n=list(self.grid.n), spacing=self.grid.spacing,
                 K=self.K, L=self.L, U=self.U, fs=self.fs, t0=self.t0, kappa=self.kappa,
                 phi_type=self.phi_type, sound_speed=self.sound_speed,
                 eir=dict(kind=self.eir.kind, fc=self.eir.fc, sigma_t=self.eir.sigma_t,
                          tc=self.eir.tc, te=self.eir.te),
                 quad_n=list(self.quad_n))
        d.update(self.meta)
        return d

    def to_json(self) -> str:
        return json.dumps(self.describe(), sort_keys=True)


# ----------------------------------------------------------------------------
# transducer arrays
# ----------------------------------------------------------------------------

def fibonacci_points(K: int, radius: float, hemisphere: bool = False) -> np.ndarray:
    j = np.arange(K, dtype=np.float64)
    z = 1.0 - (j + 0.5) / K if hemisphere else 1.0 - (2.0 * j + 1.0) / K
    phi = j * math.pi * (3.0 - math.sqrt(5.0))
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return radius * np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)


def facing_planar_array(points: np.ndarray, half_w: float, half_h: float) -> Transducers:
    """Rectangles centred at ``points`` whose normal e1 x e2 faces the origin."""
    rows = []
    for P in points:
        n = -_unit(P)
        ref = np.array([1.0, 0.0, 0.0]) if abs(n[2]) > 0.99 else np.array([0.0, 0.0, 1.0])
        e1 = _unit(np.cross(ref, n))
        e2 = np.cross(n, e1)
        rows.append(planar(P, e1, e2, half_w, half_h))
    return Transducers(np.array(rows))


def spherical_frame(P):
    r = _unit(P)
    theta = math.acos(max(-1.0, min(1.0, r[2])))
    phi = math.atan2(r[1], r[0])
    th_hat = np.array([math.cos(theta) * math.cos(phi), math.cos(theta) * math.sin(phi), -math.sin(theta)])
    ph_hat = np.array([-math.sin(phi), math.cos(phi), 0.0])
    return r, th_hat, ph_hat


def hemisphere_planar_array(K: int, radius: float, half_w: float, half_h: float) -> Transducers:
    """Rectangles on a Fibonacci hemisphere (z > 0): e1 = phi-hat (``half_w``),
    e2 = theta-hat (``half_h``), so e1 x e2 = -r-hat faces the centre."""
    rows = []
    for P in fibonacci_points(K, radius, hemisphere=True):
        _, th, ph = spherical_frame(P)
        rows.append(planar(P, ph, th, half_w, half_h))
    return Transducers(np.array(rows))


def arc_cylinder_array(n_elem: int, n_rot: int, arc_radius: float, R: float,
                       aperture_curved: float, aperture_straight: float) -> Transducers:
    """Cylindrically focused elements on a 180-degree meridian arc (polar
    angles (j + 1/2) pi / n_elem), the arc rotated ``n_rot`` times about z by
    2 pi / n_rot.  The curved (elevation) aperture is the chord
    ``aperture_curved`` (theta_max = asin(a / (2 R))); the straight aperture
    runs along the meridian tangent, which is the cylinder axis e1."""
    theta_max = math.asin(aperture_curved / (2.0 * R))
    rows = []
    for rot in range(n_rot):
        az = 2.0 * math.pi * rot / n_rot
        for j in range(n_elem):
            pol = (j + 0.5) * math.pi / n_elem
            P = arc_radius * np.array([math.sin(pol) * math.cos(az), math.sin(pol) * math.sin(az), math.cos(pol)])
            _, th, _ = spherical_frame(P)
            n = -_unit(P)
            c0 = P + R * n
            e2 = -n
            e1 = th
            rows.append(cylinder(c0, e1, e2, R, theta_max, aperture_straight / 2.0))
    return Transducers(np.array(rows))


def lib_scan_array(n_angles: int = 12, n_trans: int = 15, n_elem: int = 64, pitch: float = 0.298e-3,
                   width: float = 0.25e-3, elevation: float = 7.5e-3, R: float = 25e-3,
                   distance: float = 25e-3, sweep: float = 10e-3) -> Transducers:
    """A translate-rotate scan of a linear array with the LIB system's element
    shape (Sec. 2.6), synthesised: the measured positions are not public.

    ``n_elem`` cylindrically focused elements (focal distance R, elevation chord
    ``elevation``, width ``width`` along the array axis = the straight length)
    at ``pitch`` along z, the array facing the origin from ``distance`` in the
    xy plane; rotated to ``n_angles`` angles over 180 degrees about z and, at each
    angle, translated to ``n_trans`` positions spread over ``sweep`` along the
    tangential direction, so that the focal line sweeps across the volume.
    Transducer index = (angle * n_trans + translation) * n_elem + element."""
    theta_max = math.asin(elevation / (2.0 * R))
    rows = []
    zs = (np.arange(n_elem) - (n_elem - 1) / 2.0) * pitch
    taus = np.linspace(-sweep / 2.0, sweep / 2.0, n_trans) if n_trans > 1 else np.zeros(1)
    for a in range(n_angles):
        phi = math.pi * a / n_angles
        out = np.array([math.cos(phi), math.sin(phi), 0.0])
        tang = np.array([-math.sin(phi), math.cos(phi), 0.0])
        n = -out
        for tau in taus:
            for z in zs:
                P = distance * out + tau * tang + np.array([0.0, 0.0, z])
                rows.append(cylinder(P + R * n, [0.0, 0.0, 1.0], -n, R, theta_max, width / 2.0))
    return Transducers(np.array(rows))


# ----------------------------------------------------------------------------
# phantoms
# ----------------------------------------------------------------------------

def ball_uniform(grid: Grid, radius: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.random(grid.N)
    x = grid.coords()
    v[np.linalg.norm(x, axis=1) > radius] = 0.0
    return v


def uniform(grid: Grid, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random(grid.N)


def _subbox(grid: Grid, lo: np.ndarray, hi: np.ndarray):
    """Index ranges and coordinates of the voxels inside the box [lo, hi]."""
    rng = []
    for a in range(3):
        i0 = max(0, int(math.floor((lo[a] - grid.origin[a]) / grid.spacing)))
        i1 = min(grid.n[a] - 1, int(math.ceil((hi[a] - grid.origin[a]) / grid.spacing)))
        if i1 < i0:
            return None
        rng.append((i0, i1))
    ax = [grid.origin[a] + grid.spacing * np.arange(rng[a][0], rng[a][1] + 1) for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return rng, np.stack([X, Y, Z], axis=-1)


def _add_local(out3: np.ndarray, rng, vals: np.ndarray, op: str):
    (x0, x1), (y0, y1), (z0, z1) = rng
    view = out3[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1]
    if op == "add":
        view += vals
    else:
        np.maximum(view, vals, out=view)


def polylines(grid: Grid, rng, count: int, n_seg: int = 10, seg_len: float = 0.8e-3,
              tube_sigma: float = 0.08e-3, inner: float = 0.8) -> np.ndarray:
    """Vessel-like random walks: ``count`` polylines of ``n_seg`` segments,
    direction d <- normalize(d + 0.5 N(0, I)), tube profile exp(-d^2/(2 s^2))
    (maximum over segments), evaluated within 8 s of each segment."""
    out = np.zeros((grid.n[2], grid.n[1], grid.n[0]))
    half = np.array([(n - 1) / 2.0 * grid.spacing for n in grid.n]) * inner
    cut = 8.0 * tube_sigma
    for _ in range(count):
        p = rng.uniform(-half, half)
        d = _unit(rng.normal(size=3))
        for _s in range(n_seg):
            q = p + seg_len * d
            box = _subbox(grid, np.minimum(p, q) - cut, np.maximum(p, q) + cut)
            if box is not None:
                idx, X = box
                ab = q - p
                t = np.clip(((X - p) @ ab) / float(ab @ ab), 0.0, 1.0)
                dist2 = np.sum((X - (p + t[..., None] * ab)) ** 2, axis=-1)
                _add_local(out, idx, np.exp(-dist2 / (2.0 * tube_sigma ** 2)), "max")
            p = q
            d = _unit(d + 0.5 * rng.normal(size=3))
    return out.ravel()


def vessels(grid: Grid, rng, count: int, radius: float, n_seg: int = 10, seg_len: float = 0.8e-3,
            inner: float = 0.8) -> np.ndarray:
    """Binary vessel labels: 1 within ``radius`` of ``count`` random-walk
    polylines (the walk of ``polylines``), 0 elsewhere: a sparse support."""
    out = np.zeros((grid.n[2], grid.n[1], grid.n[0]))
    half = np.array([(n - 1) / 2.0 * grid.spacing for n in grid.n]) * inner
    for _ in range(count):
        p = rng.uniform(-half, half)
        d = _unit(rng.normal(size=3))
        for _s in range(n_seg):
            q = p + seg_len * d
            box = _subbox(grid, np.minimum(p, q) - radius, np.maximum(p, q) + radius)
            if box is not None:
                idx, X = box
                ab = q - p
                t = np.clip(((X - p) @ ab) / float(ab @ ab), 0.0, 1.0)
                dist2 = np.sum((X - (p + t[..., None] * ab)) ** 2, axis=-1)
                _add_local(out, idx, (dist2 <= radius * radius).astype(np.float64), "max")
            p = q
            d = _unit(d + 0.5 * rng.normal(size=3))
    return out.ravel()


def blobs(grid: Grid, rng, count: int, inner: float = 0.8) -> np.ndarray:
    """Sum of ``count`` Gaussian blobs: centres uniform in the inner part of the
    box, sigma ~ U[0.1, 0.4] mm, amplitude ~ U[0.2, 1], each evaluated within
    8 sigma of its centre."""
    out = np.zeros((grid.n[2], grid.n[1], grid.n[0]))
    half = np.array([(n - 1) / 2.0 * grid.spacing for n in grid.n]) * inner
    for _ in range(count):
        c = rng.uniform(-half, half)
        sig = rng.uniform(0.1e-3, 0.4e-3)
        amp = rng.uniform(0.2, 1.0)
        box = _subbox(grid, c - 8 * sig, c + 8 * sig)
        if box is None:
            continue
        idx, X = box
        d2 = np.sum((X - c) ** 2, axis=-1)
        _add_local(out, idx, amp * np.exp(-d2 / (2.0 * sig * sig)), "add")
    return out.ravel()


# ----------------------------------------------------------------------------
# window start
# ----------------------------------------------------------------------------

def transducer_circumradius(row: np.ndarray) -> float:
    if int(row[0]) == PLANAR:
        return math.hypot(row[10], row[11])
    R, th, hl = row[12], row[13], row[14]
    return math.hypot(2.0 * R * math.sin(th / 2.0), hl)


def transducer_centre(row: np.ndarray) -> np.ndarray:
    if int(row[0]) == PLANAR:
        return row[1:4].copy()
    return row[1:4] + row[12] * row[7:10]


def window_start(tr: Transducers, grid: Grid, kappa: float, c: float, fs: float,
                 margin: int = 16) -> float:
    """t0 = max(0, floor(fs (r_lo - kappa)/c) - margin)/fs with r_lo a lower
    bound of every voxel-to-surface distance (distance from the grid box to
    each transducer's bounding sphere)."""
    lo = np.array(grid.origin)
    hi = lo + (np.array(grid.n) - 1) * grid.spacing
    r_lo = math.inf
    for row in tr.packed:
        cen = transducer_centre(row)
        d = np.linalg.norm(np.maximum(0.0, np.maximum(lo - cen, cen - hi)))
        r_lo = min(r_lo, d - transducer_circumradius(row))
    n0 = max(0, int(math.floor(fs * (r_lo - kappa) / c)) - margin)
    return n0 / fs


def window_end_bound(tr: Transducers, grid: Grid, kappa: float, c: float) -> float:
    """Upper bound of every voxel-to-surface distance plus kappa."""
    corners = np.array([[grid.origin[a] + (grid.n[a] - 1) * grid.spacing * ((k >> a) & 1)
                         for a in range(3)] for k in range(8)])
    r_hi = 0.0
    for row in tr.packed:
        cen = transducer_centre(row)
        r_hi = max(r_hi, float(np.max(np.linalg.norm(corners - cen, axis=1))) + transducer_circumradius(row))
    return r_hi + kappa


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def _finish(name, tr, grid, fs, L, coef, ydraw_seed=None, U=1, quad=(16, 16), meta=None,
            phi=PHI_WENDLAND2, kappa_factor=1.5, B=None, c=SOUND_SPEED):
    kappa = kappa_factor * grid.spacing
    eir = Eir.gauss_cos()
    t0 = window_start(tr, grid, kappa, c, fs)
    coef = np.atleast_2d(np.asarray(coef, dtype=np.float64))
    y = None
    if ydraw_seed is not None:
        y = np.random.default_rng(ydraw_seed).normal(size=(coef.shape[0], tr.K, L))
    p = Problem(name, tr, grid, phi, kappa, eir, c, fs, L, U, t0, quad, coef, y, meta or {})
    end = window_end_bound(tr, grid, kappa, c) / c + eir.te
    p.meta["window_covers_signal"] = bool(end <= t0 + L / fs)
    return p


def planar64_32c(U: int = 1) -> Problem:
    """32^3 grid (0.1 mm), 64 planar 1x1 mm on a Fibonacci sphere of radius
    20 mm, fs 40 MHz, L 512; U[0,1) coefficients inside a 1.2 mm ball."""
    grid = Grid.centred(32, 0.1e-3)
    tr = facing_planar_array(fibonacci_points(64, 20e-3), 0.5e-3, 0.5e-3)
    return _finish("planar64_32c", tr, grid, 40e6, 512, ball_uniform(grid, 1.2e-3, 0), 1, U=U)


def cyl256_128c(n: int = 128, U: int = 1) -> Problem:
    """128^3 grid (0.1 mm), 256 cylinders (6 mm curved x 3 mm straight,
    R = 25 mm) on a 180-degree arc of radius 40 mm, 16 elements x 16 rotations;
    fs 50 MHz, L 2048; 200 Gaussian blobs + 16 polylines (seed 0); fine grid
    U (1 for the headline, 4 for the coarse-area-grid comparison)."""
    grid = Grid.centred(n, 0.1e-3)
    tr = arc_cylinder_array(16, 16, 40e-3, 25e-3, 6e-3, 3e-3)
    rng = np.random.default_rng(0)
    coef = blobs(grid, rng, 200) + polylines(grid, rng, 16)
    name = "cyl256_128c" if U == 1 else f"cyl256_128c_U{U}"
    return _finish(name, tr, grid, 50e6, 2048, coef, 1, U=U)


def planar512_256c(n: int = 256) -> Problem:
    """256^3 grid (0.08 mm), 512 planar 0.5x3 mm on a Fibonacci hemisphere of
    radius 50 mm, fs 50 MHz, L 4096; U[0,1) coefficients, N(0,1) signals."""
    grid = Grid.centred(n, 0.08e-3)
    tr = hemisphere_planar_array(512, 50e-3, 0.25e-3, 1.5e-3)
    return _finish("planar512_256c", tr, grid, 50e6, 4096, uniform(grid, 0), 1)


def fd_cyl8_10c() -> Problem:
    """10^3 grid (0.1 mm) with 8 cylinders of the 24x16 arc array, for the
    finite-difference check of the autograd wrapper."""
    grid = Grid.centred(10, 0.1e-3)
    full = arc_cylinder_array(24, 16, 40e-3, 25e-3, 6e-3, 3e-3)
    tr = full.subset(np.arange(0, full.K, full.K // 8)[:8])
    return _finish("fd_cyl8_10c", tr, grid, 50e6, 2048, uniform(grid, 3), 4)


def pgd_cyl384_192c(n: int = 192) -> Problem:
    """192^3 grid (0.1 mm), 384 cylinders (24 elements x 16 rotations), fs
    50 MHz, L 2048; ground truth = 24 polylines (seed 5)."""
    grid = Grid.centred(n, 0.1e-3)
    tr = arc_cylinder_array(24, 16, 40e-3, 25e-3, 6e-3, 3e-3)
    truth = polylines(grid, np.random.default_rng(5), 24)
    p = _finish("pgd_cyl384_192c", tr, grid, 50e6, 2048, truth, None)
    p.meta.update(noise_seed=6, power_seed=7, noise_level=0.01, iterations=50)
    return p


def batch8_planar256_128c(n: int = 128, B: int = 8) -> Problem:
    """B = 8 volumes on a 128^3 grid (0.1 mm), U[0,1) coefficients inside
    centred balls of sorted random radii in [0.5, 3] mm; 256 planar 1x1 mm on a
    Fibonacci sphere of radius 40 mm; fs 50 MHz, L 2048."""
    grid = Grid.centred(n, 0.1e-3)
    tr = facing_planar_array(fibonacci_points(256, 40e-3), 0.5e-3, 0.5e-3)
    radii = np.sort(np.random.default_rng(8).uniform(0.5e-3, 3e-3, size=B))
    coef = np.stack([ball_uniform(grid, float(radii[b]), 9 + b) for b in range(B)])
    p = _finish("batch8_planar256_128c", tr, grid, 50e6, 2048, coef, 1)
    p.meta["radii"] = [float(r) for r in radii]
    return p


def config_lib(n: int = 200, angles=None, translations=None, U: int = 1, vessel_count: int = 24,
               L: int = 2688) -> Problem:
    """The LIB system's scale, synthesised (Sec. 2.6): a 10 mm cube on a 200^3
    grid (50 um), the translate-rotate scan of ``lib_scan_array`` (64 elements x
    12 angles x 15 translations = 11 520 cylinders; ``angles`` / ``translations``
    select a subset), fs 62.5 MHz, L = 2688 stored samples; p0 = binary vessels
    of radius 75 um (diameter capped at three voxels) along 24 random walks
    (seed 21): ~0.3 % of the volume."""
    grid = Grid.centred(n, 10e-3 / n)
    full = lib_scan_array()
    ang = range(12) if angles is None else angles
    tra = range(15) if translations is None else translations
    idx = [(a * 15 + t) * 64 + e for a in ang for t in tra for e in range(64)]
    tr = full.subset(np.array(idx))
    coef = vessels(grid, np.random.default_rng(21), vessel_count, 75e-6)
    name = f"lib_{n}c_{tr.K}cyl" + ("" if U == 1 else f"_U{U}")
    return _finish(name, tr, grid, 62.5e6, L, coef, 22, U=U)


def small_case(shape: int = PLANAR, n: int = 6, K: int = 4, L: int = 160, fs: float = 40e6,
               U: int = 1, spacing: float = 0.1e-3, radius: float = 8e-3, seed: int = 0,
               B: int = 1, phi=PHI_WENDLAND2) -> Problem:
    """A tiny problem that the oracle finishes in well under a second.

    The array radius is scaled by an irrational factor so that no voxel-to-
    surface distance of the rational grid lands exactly on a bin edge (a
    measure-zero set on which two FP64 evaluations of the bin rule may round
    differently)."""
    radius = radius * (1.0 + math.sqrt(2.0) * 1e-3)
    grid = Grid.centred(n, spacing)
    if shape == PLANAR:
        tr = facing_planar_array(fibonacci_points(K, radius), 0.5e-3, 0.4e-3)
    else:
        full = arc_cylinder_array(8, 4, radius, 0.6 * radius, 4e-3, 2e-3)
        tr = full.subset(np.arange(0, full.K, max(1, full.K // K))[:K])
    rng = np.random.default_rng(seed)
    coef = rng.random((B, grid.N))
    p = _finish(f"small_{'pl' if shape == PLANAR else 'cy'}{K}_{n}c", tr, grid, fs, L, coef,
                seed + 1, U=U, phi=phi)
    return p


def mixed_case(n: int = 7, K_planar: int = 3, K_cyl: int = 3, L: int = 300, fs: float = 40e6, U: int = 1,
               seed: int = 0, B: int = 1) -> Problem:
    """Planar and cylindrical transducers in one array: the planar rectangles of
    ``small_case`` interleaved with the cylinders of its cylinder array (same
    irrational radius factor), so that transducer indices of the two shapes
    alternate."""
    pl = small_case(PLANAR, n=n, K=K_planar, L=L, fs=fs, U=U, seed=seed, B=B).tr.packed
    cy = small_case(CYLINDER, n=n, K=K_cyl, L=L, fs=fs, U=U, seed=seed, B=B).tr.packed
    rows = []
    for j in range(max(len(pl), len(cy))):
        if j < len(pl):
            rows.append(pl[j])
        if j < len(cy):
            rows.append(cy[j])
    tr = Transducers(np.array(rows))
    grid = Grid.centred(n, 0.1e-3)
    coef = np.random.default_rng(seed).random((B, grid.N))
    return _finish(f"mixed_pl{K_planar}_cy{K_cyl}_{n}c", tr, grid, fs, L, coef, seed + 1, U=U)


def exact_tie_case(n: int = 7, height: int = 320, L: int = 200) -> Problem:
    """Point-method distances that fall exactly on bin edges, with every
    quantity of the bin rule exact in FP64.

    Sound speed 1024 m/s and fs = 2^25 Hz make the radial step c/fs = 2^-15 m;
    the voxel spacing is one step (n odd: voxels at integer steps -(n-1)/2 ..
    (n-1)/2 on each axis), t0 is an integer number of samples, and two
    axis-aligned 8 x 8-step squares (4 x 4 points at odd integer steps) face the
    grid from ``height`` steps along +z and along +x.  Every voxel straight
    below (or beside) a point is an integer number of steps from it, so its
    arrival lies exactly on the edge between two bins; the bin rule of Alg. 2
    puts it in the upper one."""
    c, fs = 1024.0, float(2 ** 25)
    dr = c / fs
    grid = Grid.centred(n, dr)
    h = height * dr
    half = 4 * dr
    tr = Transducers(np.array([
        planar([0.0, 0.0, h], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], half, half),
        planar([h, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], half, half),
    ]))
    coef = np.random.default_rng(12).random((1, grid.N))
    p = _finish(f"exact_tie_{n}c", tr, grid, fs, L, coef, 13, quad=(4, 4), c=c)
    p.meta["tie_step"] = dr
    return p


# the full-size workloads by name (each name states its array and grid)
WORKLOADS = {f.__name__: f for f in (planar64_32c, cyl256_128c, planar512_256c, pgd_cyl384_192c,
                                      batch8_planar256_128c)}
