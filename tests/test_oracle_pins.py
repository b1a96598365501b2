"""Pins of the FP64 oracle against what the paper and mathematics fix.

The paper prints no worked numeric example, so every pin here is a closed
form, an identity, an independent library routine (scipy) or a Monte-Carlo
estimate of the plain definition |{x in Sigma : r0 <= |x - x_i| < r1}|.
Each is chosen so that a plausible mistake in the oracle (a dropped quadrant,
a wrong fold of the cylinder's angular interval, a sign in the elliptic
closed form, an off-by-one in the bin or down-sampling index) fails at least
one of them.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

import oracle as O
import pat_inputs as P
from conftest import rel_l2

C = 1500.0


# ---------------------------------------------------------------------------
# elliptic integrals (Carlson 1995; DLMF 19.36.1-2; Eq. reciprocal_modulus)
# ---------------------------------------------------------------------------

def test_carlson_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(200):
        x, y, z = rng.uniform(0, 3, 3) ** 2
        if rng.random() < 0.2:
            x = 0.0
        assert O.carlson_rf(x, y, z) == pytest.approx(sp.elliprf(x, y, z), rel=1e-14)
        assert O.carlson_rd(x, y, z + 1e-3) == pytest.approx(sp.elliprd(x, y, z + 1e-3), rel=1e-14)


@pytest.mark.parametrize("m", [0.0, 0.3, 0.9, 0.999, 1.0])
def test_ellip_e_parameter_le_one(m):
    for phi in np.linspace(0.0, math.pi / 2, 17):
        assert O.ellip_e(phi, m) == pytest.approx(sp.ellipeinc(phi, m), rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("nu", [1.02, 1.5, 3.26, 13.5])
def test_ellip_e_parameter_above_one_reciprocal_modulus(nu):
    """For nu > 1 the oracle evaluates E(theta, nu) directly with Carlson forms;
    Eq. reciprocal_modulus gives the same value from parameters below one."""
    for frac in np.linspace(0.0, 1.0, 9):
        theta = math.asin(math.sqrt(frac / nu))        # nu sin^2 theta <= 1
        tt = math.asin(min(1.0, math.sqrt(nu) * math.sin(theta)))
        ref = math.sqrt(nu) * (sp.ellipeinc(tt, 1 / nu) - (1 - 1 / nu) * sp.ellipkinc(tt, 1 / nu))
        assert O.ellip_e(theta, nu) == pytest.approx(ref, rel=1e-12, abs=1e-15)


# ---------------------------------------------------------------------------
# system kernel h (Eq. def_h, Eq. def_bh) and the temporal stage (App. C)
# ---------------------------------------------------------------------------

def _kernel_case(U=1, phi=P.PHI_WENDLAND2):
    eir = P.Eir.gauss_cos()
    kappa = 0.15e-3
    h, nf = O.build_kernel(phi, kappa, eir, C, 50e6, U)
    return h, nf, eir, kappa


def _h_cont(t, eir, kappa, phi):
    """h(t) = int g(tau) e(t - tau) dtau by adaptive quadrature (independent of the oracle)."""
    a = kappa / C

    def g(tau):
        r = C * abs(tau)
        if r >= kappa:
            return 0.0
        w = 1 - r / kappa
        return -0.5 * C * tau * (w if phi == P.PHI_CONE else w * w)

    def e(t):
        if t < 0 or t > eir.te:
            return 0.0
        d = t - eir.tc
        return math.cos(2 * math.pi * eir.fc * d) * math.exp(-d * d / (2 * eir.sigma_t ** 2))

    lo, hi = max(-a, t - eir.te), min(a, t)
    if hi <= lo:
        return 0.0
    pts = [p for p in (0.0,) if lo < p < hi]
    return si.quad(lambda tau: g(tau) * e(t - tau), lo, hi, points=pts or None, epsabs=0, epsrel=1e-12,
                   limit=200)[0]


@pytest.mark.parametrize("phi", [P.PHI_CONE, P.PHI_WENDLAND2])
def test_kernel_sums_to_zero_and_support(phi):
    """g is odd (Prop. 1), so int h = 0; the hat functions of Eq. def_bh form a
    partition of unity, so sum_n h[n] = 0.  Support as stated after
    Eq. def_downsampling."""
    h, nf, eir, kappa = _kernel_case(U=3, phi=phi)
    assert abs(h.sum()) < 1e-13 * np.abs(h).max() * len(h)
    D = 1 / (3 * 50e6)
    assert nf <= -kappa / C / D - 1 + 1e-9
    assert nf + len(h) - 1 >= (kappa / C + eir.te) / D + 1 - 1e-9


def test_kernel_taps_against_double_integral():
    """h[n] = U F_s int_0^D int_0^D h(t - t' + n D) dt dt' by nested adaptive quadrature."""
    h, nf, eir, kappa = _kernel_case(U=1, phi=P.PHI_WENDLAND2)
    D = 1 / 50e6
    hmax = np.abs(h).max()
    for n in (nf + 1, -2, 0, 5, 20, 40, nf + len(h) - 3):
        ref = si.quad(lambda s: (1 - abs(s) / D) * _h_cont(n * D + s, eir, kappa, P.PHI_WENDLAND2), -D, D,
                      points=[0.0], epsabs=1e-14 * hmax * D, epsrel=1e-11, limit=200)[0]
        assert h[n - nf] == pytest.approx(ref, abs=2e-10 * hmax)


def test_single_bin_sampling_identity():
    """App. C: for f equal to the indicator of one fine bin m0, the sampled
    signal F_s int_{t_{l-1}}^{t_l} (h * 1_bin)(t) dt equals
    1/U sum_{l'} h[U(l-1) + l' - m0] (Eq. discrete_conv, Eq. def_downsampling)."""
    U = 2
    h, nf, eir, kappa = _kernel_case(U=U, phi=P.PHI_CONE)
    fs = 50e6
    D = 1 / (U * fs)
    m0 = 7
    hmax = np.abs(h).max()
    for l in (4, 6, 8, 12, 20):
        disc = sum(h[U * (l - 1) + lp - m0 - nf] for lp in range(1, U + 1)
                   if 0 <= U * (l - 1) + lp - m0 - nf < len(h)) / U
        t_lo, t_hi = (l - 1) / fs, l / fs          # t0 = 0

        def inner(t):
            # (h * 1_[tau_{m0-1}, tau_{m0}))(t) = int_{tau_{m0-1}}^{tau_{m0}} h(t - t') dt'
            return si.quad(lambda tp: _h_cont(t - tp, eir, kappa, P.PHI_CONE), (m0 - 1) * D, m0 * D,
                           epsabs=0, epsrel=1e-10, limit=100)[0]
        cont = fs * si.quad(inner, t_lo, t_hi, epsabs=1e-14 * hmax * D, epsrel=1e-9, limit=100)[0]
        assert disc == pytest.approx(cont, rel=1e-9, abs=1e-9 * hmax)


def test_temporal_stage_matches_numpy_convolution():
    """s_hat = D_U(h * f) of the oracle equals numpy's convolution of its own f."""
    p = P.small_case(P.PLANAR, n=5, K=2, U=3, L=150)
    h, nf = O.kernel_of(p)
    s = O.forward(p, kernel=(h, nf))
    for k in range(p.K):
        f, Mlo = O.fcoef(p, k, kernel=(h, nf))
        full = np.convolve(f[0], h)                  # index i <-> fine bin Mlo + nf + i
        first = Mlo + nf
        U, L = p.U, p.L
        ref = np.array([sum(full[U * (l - 1) + lp - first] for lp in range(1, U + 1)) / U
                        for l in range(1, L + 1)])
        assert rel_l2(s[0, k], ref) < 1e-13


# ---------------------------------------------------------------------------
# shell areas (Alg. 4) against the plain definition
# ---------------------------------------------------------------------------

def _planar_area_by_v(tr, x, r0, r1):
    """|{(u, v) in rect : r0^2 <= u^2 + v^2 + z^2 < r1^2}| integrating the u-length over v."""
    e1, e2, c0 = tr[4:7], tr[7:10], tr[1:4]
    n3 = np.cross(e1, e2)
    d = x - c0
    x1, x2, x3 = d @ e1, d @ e2, d @ n3
    L1, L2 = tr[10], tr[11]

    def ulen(v):
        def meas(rr):   # |{u in [-L1 - x1, L1 - x1] : u^2 < rr^2 - v^2 - x3^2}|
            q = rr * rr - v * v - x3 * x3
            if q <= 0:
                return 0.0
            w = math.sqrt(q)
            return max(0.0, min(w, L1 - x1) - max(-w, -L1 - x1))
        return meas(r1) - meas(r0)

    lo, hi = -L2 - x2, L2 - x2
    pts = []
    for rr in (r0, r1):
        q = rr * rr - x3 * x3
        for u in (-L1 - x1, L1 - x1, 0.0):
            if q - u * u > 0:
                pts += [math.sqrt(q - u * u), -math.sqrt(q - u * u)]
    pts = sorted(p for p in pts if lo < p < hi)
    return si.quad(ulen, lo, hi, points=pts or None, epsabs=1e-16, epsrel=1e-12, limit=400)[0]


def _cyl_area_by_v(tr, x, r0, r1):
    """Cylinder: integrate over the axial coordinate the angular measure of the
    surface points at distance in [r0, r1), times R (the surface element R dtheta dz)."""
    e1, e2, c0 = tr[4:7], tr[7:10], tr[1:4]
    n3 = np.cross(e1, e2)
    d = x - c0
    x1, x2, x3 = d @ e2, d @ n3, d @ e1
    R, th, Lz = tr[12], tr[13], tr[14]
    rho = math.hypot(x1, x2)
    thi = math.atan2(x2, x1)

    def ang(v):
        # theta in [-th, th] with rho^2 + R^2 - 2 R rho cos(theta - thi) in [r0^2 - v^2, r1^2 - v^2)
        def meas(rr):
            q = rr * rr - v * v
            if rho == 0.0:
                return 2 * th if R * R < q else 0.0
            cval = (rho * rho + R * R - q) / (2 * R * rho)  # cos(theta - thi) > cval
            if cval >= 1:
                return 0.0
            if cval <= -1:
                return 2 * th
            a = math.acos(cval)
            tot = 0.0
            for k in (-1, 0, 1):
                lo2, hi2 = thi - a + 2 * math.pi * k, thi + a + 2 * math.pi * k
                tot += max(0.0, min(hi2, th) - max(lo2, -th))
            return tot
        return meas(r1) - meas(r0)

    lo, hi = -Lz - x3, Lz - x3
    # kinks of the integrand: an arc end crossing an aperture edge or a fold point
    pts = [0.0]
    for rr in (r0, r1):
        for phi in (th - thi, -th - thi, 0.0, math.pi):
            q = rr * rr - (rho * rho + R * R - 2 * R * rho * math.cos(phi))
            if q > 0:
                pts += [math.sqrt(q), -math.sqrt(q)]
    pts = sorted(p for p in pts if lo < p < hi)
    return R * si.quad(ang, lo, hi, points=pts or None, epsabs=1e-17, epsrel=1e-13, limit=800)[0]


def _random_planar(rng):
    n = P._unit(rng.normal(size=3))
    c0 = -6e-3 * n
    ref = np.array([1.0, 0, 0]) if abs(n[2]) > 0.9 else np.array([0, 0, 1.0])
    e1 = P._unit(np.cross(ref, n))
    e2 = np.cross(n, e1)
    return P.planar(c0, e1, e2, rng.uniform(0.2e-3, 1.5e-3), rng.uniform(0.2e-3, 1.5e-3))


def _random_cyl(rng):
    n = P._unit(rng.normal(size=3))
    P0 = -8e-3 * n
    R = rng.uniform(4e-3, 12e-3)
    ax = P._unit(np.cross(n, P._unit(rng.normal(size=3))))
    return P.cylinder(P0 + R * n, ax, -n, R, rng.uniform(0.1, 1.2), rng.uniform(0.3e-3, 2e-3))


@pytest.mark.parametrize("seed", range(6))
def test_planar_shell_area_matches_definition(seed):
    rng = np.random.default_rng(seed)
    tr = _random_planar(rng)
    x = rng.uniform(-2e-3, 2e-3, 3)
    l0, a = O.pair_areas(tr, x, C, 0.0, 40e6)
    dr = C / 40e6
    tot = 4 * tr[10] * tr[11]
    for j in range(0, len(a), max(1, len(a) // 12)):
        r0, r1 = (l0 + j - 1) * dr, (l0 + j) * dr
        assert a[j] == pytest.approx(_planar_area_by_v(tr, x, r0, r1), abs=1e-10 * tot)
    assert a.sum() == pytest.approx(tot, rel=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_cylinder_shell_area_matches_definition(seed):
    rng = np.random.default_rng(100 + seed)
    tr = _random_cyl(rng)
    x = rng.uniform(-2e-3, 2e-3, 3)
    if seed == 0:   # a voxel behind the focal line (angular interval wraps through pi)
        x = tr[1:4] - 3e-3 * tr[7:10] + 0.2e-3 * np.cross(tr[4:7], tr[7:10])
    l0, a = O.pair_areas(tr, x, C, 0.0, 50e6)
    dr = C / 50e6
    tot = 2 * tr[13] * tr[12] * 2 * tr[14]
    for j in range(0, len(a), max(1, len(a) // 12)):
        r0, r1 = (l0 + j - 1) * dr, (l0 + j) * dr
        assert a[j] == pytest.approx(_cyl_area_by_v(tr, x, r0, r1), abs=1e-9 * tot)
    assert a.sum() == pytest.approx(tot, rel=1e-13)


def test_shell_areas_against_monte_carlo():
    rng = np.random.default_rng(7)
    tr = P.planar([0, 0, 5e-3], [1, 0, 0], [0, 1, 0], 0.5e-3, 0.4e-3)
    x = np.array([0.2e-3, -0.1e-3, 0.0])
    n = 2_000_000
    uv = rng.uniform([-0.5e-3, -0.4e-3], [0.5e-3, 0.4e-3], size=(n, 2))
    d = np.sqrt((uv[:, 0] - x[0]) ** 2 + (uv[:, 1] - x[1]) ** 2 + (5e-3 - x[2]) ** 2)
    A = 0.8e-6
    l0, a = O.pair_areas(tr, x, C, 0.0, 40e6)
    dr = C / 40e6
    hist = np.histogram(d, bins=(np.arange(l0 - 1, l0 + len(a))) * dr)[0]
    mc = A * hist / n
    sd = A * np.sqrt(np.maximum(hist, 1)) / n
    assert np.all(np.abs(a - mc) < 5 * sd)


def test_planar_on_axis_annulus():
    """Voxel on the rectangle's normal axis: while the annulus fits inside the
    rectangle, |M^l| = pi (r_l^2 - r_{l-1}^2) and f_i[l] = 2 pi c exactly
    (r_l^2 - r_{l-1}^2 = 2 r_{l-1/2} dr; the constant on-axis SIR of the remark
    on the connection with the SIR)."""
    tr = P.planar([0, 0, 0], [1, 0, 0], [0, 1, 0], 3.0e-3, 2.5e-3)
    z = 4e-3
    x = np.array([0.0, 0.0, z])
    fs = 40e6
    dr = C / fs
    l0, a = O.pair_areas(tr, x, C, 0.0, fs)
    rmax_inside = math.sqrt(z * z + 2.5e-3 ** 2)
    checked = 0
    for j, area in enumerate(a):
        r0, r1 = (l0 + j - 1) * dr, (l0 + j) * dr
        if r1 > rmax_inside:
            break
        if r0 < z:
            assert area == pytest.approx(math.pi * (r1 * r1 - z * z), rel=1e-12)
        else:
            assert area == pytest.approx(math.pi * (r1 * r1 - r0 * r0), rel=1e-12)
            assert fs * area / (C * (l0 + j - 0.5) / fs) == pytest.approx(2 * math.pi * C, rel=1e-12)
            checked += 1
    assert checked >= 3


def test_cylinder_on_focal_line():
    """rho = 0 (voxel on the focal line): every surface point is at distance
    sqrt(R^2 + v^2), so |M^l| = 2 theta_max R |{v : R^2 + v^2 in [r_{l-1}^2, r_l^2)}|."""
    R, th, Lz = 10e-3, 0.4, 1.5e-3
    tr = P.cylinder([0, 0, 0], [0, 0, 1], [1, 0, 0], R, th, Lz)
    x = np.array([0.0, 0.0, 0.6e-3])
    fs = 50e6
    dr = C / fs
    l0, a = O.pair_areas(tr, x, C, 0.0, fs)
    v1, v2 = -Lz - x[2], Lz - x[2]

    def vmeas(r):
        if r <= R:
            return 0.0
        w = math.sqrt(r * r - R * R)
        return max(0.0, min(w, v2) - max(-w, v1))
    for j, area in enumerate(a):
        r0, r1 = (l0 + j - 1) * dr, (l0 + j) * dr
        assert area == pytest.approx(2 * th * R * (vmeas(r1) - vmeas(r0)), rel=1e-12, abs=1e-13 * R * Lz)


def test_point_transducer_limit():
    """A transducer shrunk far below one radial step lies in a single bin: the
    surface coefficient |Sigma|/(c tau_{m-1/2}) and the point coefficient
    dA/r summed over its points differ only by the ratio r/(c tau_{m-1/2})."""
    p = P.small_case(P.PLANAR, n=3, K=2, L=160)
    p.tr.packed[:, 10] = 2e-7
    p.tr.packed[:, 11] = 1.5e-7
    p.quad_n = (2, 2)
    h, nf = O.kernel_of(p)
    for k in range(p.K):
        fs_, Mlo = O.fcoef(p, k, mode=O.MODE_SURFACE, kernel=(h, nf))
        fp_, _ = O.fcoef(p, k, mode=O.MODE_POINT, kernel=(h, nf))
        m = np.nonzero(fs_[0])[0]
        # every bin is hit by both methods, with nearly the same weight
        assert np.array_equal(m, np.nonzero(fp_[0])[0]) or rel_l2(fp_, fs_) < 1e-3
        assert rel_l2(fp_, fs_) < 2e-3


def _rotated_frame(seed):
    """Orthonormal e1, e2 of a random orientation and their normal e1 x e2."""
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q[:, 0], q[:, 1], np.cross(q[:, 0], q[:, 1])


@pytest.mark.parametrize("shape", [P.PLANAR, P.CYLINDER])
def test_quadrature_points_are_cell_centres_on_the_surface(shape):
    """Alg. 2 with the tensor midpoint rule (Prop. 2: barycentres of equal
    cells of the parameter rectangle D): every point lies on the surface of
    Eq. plane_param / Eq. cylinder_param, the points are exactly the cell
    centres of the n1 x n2 partition of D, each once, and Q dA is the area of
    the surface (R 2 theta_max 2 L_z for the cylinder, whose area element is
    R du dv)."""
    e1, e2, n3 = _rotated_frame(5 + shape)
    c0 = np.array([1.3e-3, -2.1e-3, 0.7e-3])
    n1, n2 = 7, 5
    if shape == P.PLANAR:
        L1, L2 = 0.6e-3, 0.35e-3
        tr = P.planar(c0, e1, e2, L1, L2)
        area = 4 * L1 * L2
    else:
        R, th, Lz = 9e-3, 0.37, 1.2e-3
        tr = P.cylinder(c0, e1, e2, R, th, Lz)
        area = 2 * th * R * 2 * Lz
    pts, dA = O.quad_points(tr, n1, n2)
    assert pts.shape == (n1 * n2, 3)
    assert n1 * n2 * dA == pytest.approx(area, rel=1e-14)
    d = pts - c0
    if shape == P.PLANAR:
        u, v = d @ e1, d @ e2
        assert np.max(np.abs(d @ n3)) < 1e-15            # in the plane of the rectangle
        cu = -L1 + (np.arange(n1) + 0.5) * 2 * L1 / n1
        cv = -L2 + (np.arange(n2) + 0.5) * 2 * L2 / n2
    else:
        z = d @ e1
        radial = d - np.outer(z, e1)
        # on the cylinder of radius R about the focal line through c0 along e1
        assert np.max(np.abs(np.linalg.norm(radial, axis=1) / R - 1.0)) < 1e-14
        # angle from e2 about the axis; the sign of e1 x e2 is immaterial
        # (reading 13), so the cell centres are compared up to that sign
        u = np.arctan2(radial @ n3, radial @ e2)
        v = z
        assert np.max(np.abs(u)) < th
        cu = -th + (np.arange(n1) + 0.5) * 2 * th / n1
        cv = -Lz + (np.arange(n2) + 0.5) * 2 * Lz / n2
    grid = {(a, b) for a in range(n1) for b in range(n2)}
    got = set()
    for uu, vv in zip(u, v):
        a = int(np.argmin(np.abs(cu - uu)))
        b = int(np.argmin(np.abs(cv - vv)))
        assert abs(cu[a] - uu) < 1e-12 * max(1.0, abs(cu[0])) and abs(cv[b] - vv) < 1e-15
        got.add((a, b))
    assert got == grid


@pytest.mark.parametrize("shape", [P.PLANAR, P.CYLINDER])
def test_single_voxel_point_transducer_limit_is_exact(shape):
    """One voxel and a transducer far below one radial step: its whole
    surface falls in the bin m holding the distance r to the surface centre,
    and the two methods reduce to their definitions (Eq. ui_area,
    Eq. def_f_point): the surface coefficient is U F_s |Sigma| / (c tau_{m-1/2})
    exactly and the point coefficient U F_s sum_j dA_j / r_j tends to
    U F_s |Sigma| / r (second order in the patch size with centred points).
    A misplaced point set (another part of the cylinder, the axis or the
    back of the focal line) lands in another bin; a cell area without the
    cylinder's R scales the value."""
    p = P.small_case(shape, n=1, K=3, L=300)
    p.coef = np.ones((1, 1))
    tr = p.tr.packed
    if shape == P.CYLINDER:
        tr[:, 13], tr[:, 14] = 2e-5, 1.5e-7
        area = 2 * tr[:, 13] * tr[:, 12] * 2 * tr[:, 14]
        centre = tr[:, 1:4] + tr[:, 12:13] * tr[:, 7:10]   # surface point at angle 0
    else:
        tr[:, 10], tr[:, 11] = 2e-7, 1.5e-7
        area = 4 * tr[:, 10] * tr[:, 11]
        centre = tr[:, 1:4]
    p.quad_n = (2, 2)
    h, nf = O.kernel_of(p)
    ufs, c = p.U * p.fs, p.sound_speed
    for k in range(p.K):
        f_surf, Mlo = O.fcoef(p, k, mode=O.MODE_SURFACE, kernel=(h, nf))
        f_pt, Mlo2 = O.fcoef(p, k, mode=O.MODE_POINT, kernel=(h, nf))
        assert Mlo == Mlo2
        nz_s, nz_p = np.nonzero(f_surf[0])[0], np.nonzero(f_pt[0])[0]
        assert len(nz_s) == 1 and np.array_equal(nz_s, nz_p)
        m = Mlo + int(nz_s[0])
        r = float(np.linalg.norm(centre[k] - np.asarray(p.grid.origin)))
        assert c * (p.t0 + (m - 1) / ufs) <= r < c * (p.t0 + m / ufs)     # bin rule of Alg. 2
        assert f_surf[0, nz_s[0]] == pytest.approx(ufs * area[k] / (c * (p.t0 + (m - 0.5) / ufs)), rel=1e-10)
        assert f_pt[0, nz_p[0]] == pytest.approx(ufs * area[k] / r, rel=1e-9)


def test_cylinder_point_method_converges_to_surface_method():
    """Prop. 2 on the cylinder (Sec. 4.2 parametrisation): with the bin grid
    fixed, the point method's coefficients tend to the exact cell averages of
    1/r, which the surface method equals up to its midpoint rule (~1e-7 here),
    so the signals converge to the surface method's.  While the smooth part of
    the quadrature error dominates, it falls as Q^-1 (a factor ~4 per doubling
    of n1 = n2); later the arrival-time jumps between bins slow it.  A
    left-point rule (first order, a factor ~2), points on the wrong side of the
    focal line or a cell area without R do not converge to it."""
    p = P.small_case(P.CYLINDER, n=3, K=2, L=300, U=4)
    h, nf = O.kernel_of(p)
    s_surf = O.forward(p, kernel=(h, nf))
    qs = [2, 4, 8, 16, 32, 64, 128]
    errs = []
    for q in qs:
        p.quad_n = (q, q)
        errs.append(rel_l2(O.forward(p, mode=O.MODE_POINT, kernel=(h, nf)), s_surf))
    for a, b in zip(errs[:3], errs[1:4]):
        assert a / b > 3.0, errs
    slope = np.polyfit(np.log(np.array(qs, dtype=float) ** 2), np.log(errs), 1)[0]
    assert slope < -0.6, (slope, errs)
    assert errs[-1] < 2e-3


# ---------------------------------------------------------------------------
# operator identities
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [P.PLANAR, P.CYLINDER])
@pytest.mark.parametrize("mode", [O.MODE_SURFACE, O.MODE_POINT])
@pytest.mark.parametrize("U", [1, 3])
def test_dot_product(shape, mode, U):
    """<A p0, y> = <p0, A^T y> (appendix on adjoint operators) to rounding."""
    p = P.small_case(shape, n=5, K=3, U=U, L=300 if shape == P.CYLINDER else 160, B=2)
    p.quad_n = (5, 4)
    s = O.forward(p, mode=mode)
    z = O.adjoint(p, mode=mode)
    lhs, rhs = np.sum(s * p.y), np.sum(z * p.coef)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(s) * np.linalg.norm(p.y) * 1e-3)


def test_rotation_covariance():
    """Rotating transducers by 90 degrees about z and the coefficients with them
    (the centred grid maps to itself) leaves every signal unchanged."""
    p = P.small_case(P.CYLINDER, n=6, K=3, L=300)
    s = O.forward(p)
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]])
    q = P.small_case(P.CYLINDER, n=6, K=3, L=300)
    for row in q.tr.packed:
        for a in (1, 4, 7):
            row[a:a + 3] = Rz @ row[a:a + 3]
    n = p.grid.n[0]
    c = p.coef[0].reshape(n, n, n)              # [iz, iy, ix]
    # voxel (ix, iy) moves to (n-1-iy, ix): new[iz, iy', ix'] = old[iz, ix', n-1-iy']
    cr = np.transpose(c, (0, 2, 1))[:, :, ::-1]
    s2 = O.forward(q, coef=cr.reshape(1, -1))
    assert rel_l2(s2, s) < 1e-13


def test_linearity():
    p = P.small_case(P.PLANAR, n=5, K=2, L=160, B=2)
    a = O.forward(p, coef=p.coef[:1])
    b = O.forward(p, coef=p.coef[1:])
    ab = O.forward(p, coef=(2.0 * p.coef[:1] - 0.5 * p.coef[1:]))
    assert rel_l2(ab, 2.0 * a - 0.5 * b) < 1e-13


def test_surface_converges_to_point_with_many_points():
    """Prop. 2 / Prop. 3: as the quadrature is refined the point method
    approaches the surface method up to the midpoint error of 1/r; the
    difference drops with Q and levels off."""
    p = P.small_case(P.PLANAR, n=3, K=2, L=160)
    h, nf = O.kernel_of(p)
    fsurf = O.forward(p, kernel=(h, nf))
    errs = []
    for q in (2, 4, 8, 16, 32):
        p.quad_n = (q, q)
        errs.append(rel_l2(O.forward(p, mode=O.MODE_POINT, kernel=(h, nf)), fsurf))
    assert errs[-1] < errs[0] / 10
    assert errs[-1] < 0.05


def test_point_bin_rule_on_exact_ties():
    """Alg. 2's bin rule l = floor((r/c - t0) U F_s) + 1 on distances that lie
    exactly on bin edges (reading 1: half-open bins, a distance on an edge goes
    to the upper bin), against brute force in exact integer arithmetic: in the
    exact-tie workload every distance is sqrt of an integer number of squared
    radial steps, so floor(r / dr) = isqrt(r^2 / dr^2) with no rounding."""
    p = P.exact_tie_case()
    dr = p.meta["tie_step"]
    ufs = p.U * p.fs
    r0 = int(round(p.t0 * ufs))
    assert r0 == p.t0 * ufs
    n = p.grid.n[0]
    h, nf = O.kernel_of(p)
    ties = 0
    for k in range(p.K):
        f_or, Mlo = O.fcoef(p, k, mode=O.MODE_POINT, kernel=(h, nf))
        pts, dA = O.quad_points(p.tr.packed[k], *p.quad_n)
        ip = np.rint(pts / dr).astype(np.int64)
        assert np.array_equal(ip * dr, pts)               # points on the integer lattice of dr
        f = np.zeros_like(f_or)
        for i in range(p.N):
            vox = np.array([i % n, (i // n) % n, i // (n * n)]) - (n - 1) // 2
            for q in ip:
                r2 = int(np.sum((q - vox) ** 2))
                s = math.isqrt(r2)
                ties += s * s == r2
                m = s - r0 + 1                              # floor(r/dr - r0) + 1
                f[0, m - Mlo] += p.coef[0, i] * dA / (math.sqrt(r2) * dr)
        f *= ufs
        assert rel_l2(f_or, f) < 1e-14
        assert np.max(np.abs(f_or - f)) <= 1e-13 * np.max(np.abs(f))
    assert ties >= 2 * 16 * n
