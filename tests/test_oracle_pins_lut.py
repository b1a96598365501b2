"""Pins of the oracle's lookup-table I_l (Sec. 4.2, LUT paragraph).

The tables hold E~(s, nu) = E(arcsin s, nu) and F~(s, nu) = F(arcsin s, nu) on
the power-law grid of Eq. LUT_sampling (1000 x 1000, exponent 4, eps = 1e-16);
a query interpolates bilinearly, and nu > 1 goes through the
reciprocal-modulus transformation (Eq. reciprocal_modulus).

Pinned against scipy's incomplete elliptic integrals (the node values), closed
forms on the axes (E~(s, 0) = F~(s, 0) = arcsin s; zero at s = 0), Gauss-Legendre
quadrature of the integrand for nu > 1, second-order convergence of the
bilinear interpolation as the grid is refined (a wrong weight, index or grid
inversion breaks it), exact reproduction at the nodes, and at the level of the
areas: conservation of the total area (the I_l telescope), convergence to the
exact areas, planar transducers untouched and the adjoint identity.
"""
import math

import numpy as np
import pytest
from scipy.special import ellipeinc, ellipkinc

import oracle as O
import pat_inputs as P
from conftest import rel_l2

C = P.SOUND_SPEED


@pytest.fixture(autouse=True)
def _default_size():
    O.lut_set_size(O.LUT_SIZE)
    yield
    O.lut_set_size(O.LUT_SIZE)


def _gl_e(theta, nu, n=200):
    """E(theta, nu) by n-point Gauss-Legendre on [0, theta] (smooth integrand
    while nu sin^2 theta < 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * theta * (x + 1.0)
    return 0.5 * theta * np.sum(w * np.sqrt(1.0 - nu * np.sin(t) ** 2))


def test_grid_nodes_follow_the_power_law():
    N = O.LUT_SIZE
    s0, n0, _, _ = O.lut_entry(0, 0)
    s1, n1, _, _ = O.lut_entry(N - 1, N - 1)
    assert s0 == 0.0 and n0 == 0.0
    assert s1 == 1.0 - 1e-16 and n1 == 1.0 - 1e-16 and s1 < 1.0
    xs = np.array([O.lut_entry(i, 0)[0] for i in range(N)])
    assert np.all(np.diff(xs) > 0)
    # exponent 4: the gaps shrink like (1 - t)^3 towards the singular corner
    assert (1.0 - xs[N - 2]) == pytest.approx((1.0 / (N - 1)) ** 4, rel=1e-3)
    assert xs[1] == pytest.approx(4.0 / (N - 1), rel=1e-2)


def test_axes_are_closed_forms():
    N = O.LUT_SIZE
    for i in range(0, N, 37):
        s, nu, E, F = O.lut_entry(i, 0)
        assert nu == 0.0
        assert E == pytest.approx(math.asin(s), rel=1e-14, abs=1e-300)
        assert F == pytest.approx(math.asin(s), rel=1e-14, abs=1e-300)
        s, nu, E, F = O.lut_entry(0, i)
        assert s == 0.0 and E == 0.0 and F == 0.0


def test_nodes_hold_the_elliptic_integrals():
    rng = np.random.default_rng(3)
    N = O.LUT_SIZE
    idx = list(zip(rng.integers(1, N - 1, 300), rng.integers(0, N - 1, 300)))
    idx += [(N - 2, 500), (700, N - 2), (1, 1), (N - 3, N - 3)]
    worst = 0.0
    for i, j in idx:
        s, nu, E, F = O.lut_entry(int(i), int(j))
        th = math.atan2(s, math.sqrt((1.0 - s) * (1.0 + s)))
        # the amplitude near pi/2 carries a rounding of ~1e-16 / sqrt(1 - nu s^2)
        # relative to itself through dF/dtheta; keep the comparison where that is small
        if 1.0 - nu * s * s < 1e-10:
            continue
        worst = max(worst, abs(E - ellipeinc(th, nu)) / E, abs(F - ellipkinc(th, nu)) / F)
    assert worst < 1e-11


def test_singular_corner_is_finite_and_e_tends_to_one():
    N = O.LUT_SIZE
    s, nu, E, F = O.lut_entry(N - 1, N - 1)
    assert E == pytest.approx(1.0, abs=1e-12)          # E(pi/2, 1) = 1
    assert math.isfinite(F) and 15.0 < F < 25.0        # logarithmic growth of F(pi/2, nu -> 1)


def test_lookup_reproduces_the_nodes():
    """At a node the interpolation returns the stored value (the weights are
    linear in the coordinates, so a node found in either neighbouring cell
    gives it)."""
    for i, j in [(3, 5), (500, 640), (998, 2), (10, 997), (999, 999), (999, 0), (900, 998)]:
        s, nu, E, _ = O.lut_entry(i, j)
        assert O.lut_e(s, nu) == pytest.approx(E, rel=1e-13, abs=1e-15)


def _lookup_error(N, pts):
    O.lut_set_size(N)
    return max(abs(O.lut_e(math.sin(th), nu) - ref) for th, nu, ref in pts)


def test_bilinear_interpolation_is_second_order():
    rng = np.random.default_rng(8)
    pts = []
    for _ in range(400):
        th, nu = rng.uniform(0.0, 1.4), rng.uniform(0.0, 0.95)
        pts.append((th, nu, float(ellipeinc(th, nu))))
    errs = [_lookup_error(N, pts) for N in (126, 251, 501, 1001)]
    assert errs[-1] < 2e-6, errs
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 5.0, errs


def test_reciprocal_modulus_branch():
    """nu > 1 with nu sin^2 theta <= 0.9 (Lemma exact_integral keeps
    nu sin^2 theta <= 1 for the cylinder), against Gauss-Legendre quadrature."""
    rng = np.random.default_rng(12)
    pts = []
    for _ in range(200):
        nu = math.exp(rng.uniform(0.01, 4.0))
        th = math.asin(math.sqrt(rng.uniform(0.0, 0.9) / nu))
        pts.append((th, nu, _gl_e(th, nu)))
    errs = [_lookup_error(N, pts) for N in (251, 501, 1001)]
    assert errs[-1] < 2e-5, errs
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 5.0, errs


def _cyl(th=0.3, R=10e-3, Lz=1.2e-3):
    return P.cylinder([0, 0, 0], [0, 0, 1], [1, 0, 0], R, th, Lz)


@pytest.mark.parametrize("seed", range(4))
def test_lut_areas_conserve_the_total_area(seed):
    """The I_l of consecutive edges telescope: the tables change how the area is
    split over the bins, never its total."""
    rng = np.random.default_rng(70 + seed)
    tr = _cyl(th=rng.uniform(0.1, 0.6))
    x = rng.uniform(-2e-3, 2e-3, 3)
    _, a = O.pair_areas_mode(tr, x, C, 0.0, 50e6, O.MODE_LUT, 1)
    assert a.sum() == pytest.approx(2 * tr[13] * tr[12] * 2 * tr[14], rel=1e-12)


def test_lut_areas_converge_to_the_exact_areas():
    rng = np.random.default_rng(5)
    tr = _cyl(th=0.45)
    xs = [rng.uniform(-2e-3, 2e-3, 3) for _ in range(6)]
    exact = [O.pair_areas(tr, x, C, 0.0, 50e6)[1] for x in xs]
    errs = []
    for N in (251, 501, 1001):
        O.lut_set_size(N)
        d = sum(np.abs(O.pair_areas_mode(tr, x, C, 0.0, 50e6, O.MODE_LUT, 1)[1] - e).sum()
                for x, e in zip(xs, exact))
        errs.append(d / sum(np.abs(e).sum() for e in exact))
    assert 0 < errs[-1] < 2e-4, errs
    assert errs[0] / errs[-1] > 6.0, errs


def test_lut_leaves_planar_transducers_exact():
    p = P.small_case(P.PLANAR, n=4, K=2, L=160)
    assert rel_l2(O.forward(p, mode=O.MODE_LUT), O.forward(p)) < 1e-14


def test_lut_operator_is_adjoint_and_close_to_exact():
    p = P.small_case(P.CYLINDER, n=5, K=3, U=2, L=300, B=2)
    s = O.forward(p, mode=O.MODE_LUT)
    z = O.adjoint(p, mode=O.MODE_LUT)
    lhs, rhs = np.sum(s * p.y), np.sum(z * p.coef)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(s) * np.linalg.norm(p.y)
    e = rel_l2(s, O.forward(p))
    assert 0 < e < 1e-3
