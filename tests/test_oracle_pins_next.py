"""Pins of the oracle's two approximate surface variants.

Coarse area grid (Remark 1): the area of each shell of `step` fine bins, split
evenly over its bins.  Pinned by the single-shell closed form over the coarse
radii (an independent evaluation: two edges of Alg. 4 instead of a sum of
fine bins), equality inside each shell, alignment of the shells, conservation
of the total area, step = 1 reducing to the exact method, and the adjoint
identity of the operator built on it.

Trapezoidal I_l (Eq. trapezoid_Il, cylinder): exact when the level curve is
flat in the angle (voxel on the focal line), total area conserved (I_l
vanishes at both ends of every sweep), error vanishing as the angular
aperture shrinks at the rate of a trapezoid rule (second order), and planar
transducers untouched.
"""
import math

import numpy as np
import pytest

import oracle as O
import pat_inputs as P
from conftest import rel_l2

C = P.SOUND_SPEED


def _cyl(th=0.3, R=10e-3, Lz=1.2e-3):
    return P.cylinder([0, 0, 0], [0, 0, 1], [1, 0, 0], R, th, Lz)


def _tot_cyl(tr):
    return 2 * tr[13] * tr[12] * 2 * tr[14]


# ---------------------------------------------------------------------------
# coarse area grid
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [P.PLANAR, P.CYLINDER])
@pytest.mark.parametrize("step", [2, 3, 5])
def test_coarse_shells_match_single_shell_closed_form(shape, step):
    rng = np.random.default_rng(11 + step)
    if shape == P.PLANAR:
        tr = P.planar([0, 0, 5e-3], [1, 0, 0], [0, 1, 0], 0.9e-3, 0.6e-3)
        tot = 4 * tr[10] * tr[11]
    else:
        tr = _cyl()
        tot = _tot_cyl(tr)
    x = rng.uniform(-1.5e-3, 1.5e-3, 3)
    fs, t0 = 40e6 * step, 1.1e-7
    ufs = fs
    l0, a = O.pair_areas_mode(tr, x, C, t0, ufs, O.MODE_SURFACE, step)
    lf, af = O.pair_areas_mode(tr, x, C, t0, ufs, O.MODE_SURFACE, 1)
    assert (l0 - 1) % step == 0 and len(a) % step == 0, "shells start at bins 1 (mod step)"
    assert a.sum() == pytest.approx(tot, rel=1e-12)
    assert a.sum() == pytest.approx(af.sum(), rel=1e-13)
    for s in range(0, len(a), step):
        shell = a[s:s + step]
        assert np.all(shell == shell[0]), "a shell's area is split evenly"
        j_last = l0 + s + step - 1
        r0 = C * (t0 + (j_last - step) / ufs)
        r1 = C * (t0 + j_last / ufs)
        ref = O.shell_area(tr, x, r0, r1)
        assert shell.sum() == pytest.approx(ref, abs=1e-12 * tot)


def test_step_one_is_the_exact_method():
    tr = _cyl()
    x = np.array([0.4e-3, -0.7e-3, 0.2e-3])
    l0, a = O.pair_areas_mode(tr, x, C, 0.0, 50e6, O.MODE_SURFACE, 1)
    l1, b = O.pair_areas(tr, x, C, 0.0, 50e6)
    assert l0 == l1 and np.array_equal(a, b)
    p = P.small_case(P.CYLINDER, n=4, K=2, U=2, L=300)
    s1 = O.forward(p, step=1)
    s0 = O.forward(p, step=None)
    assert rel_l2(s1, s0) < 1e-14    # equal up to the order of the threads' partial sums


@pytest.mark.parametrize("shape", [P.PLANAR, P.CYLINDER])
def test_coarse_grid_operator_is_adjoint(shape):
    p = P.small_case(shape, n=5, K=3, U=3, L=300 if shape == P.CYLINDER else 200, B=2)
    p.area_step = 3
    s = O.forward(p)
    z = O.adjoint(p)
    lhs, rhs = np.sum(s * p.y), np.sum(z * p.coef)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(s) * np.linalg.norm(p.y)
    exact = O.forward(p, step=1)
    # an approximation of the exact operator, not the exact operator itself
    e = rel_l2(s, exact)
    assert 0 < e < 0.5


# ---------------------------------------------------------------------------
# trapezoidal I_l
# ---------------------------------------------------------------------------

def test_trapezoid_exact_on_the_focal_line():
    """rho = 0: Psi(u, r) does not depend on the angle, so the chord is the curve."""
    tr = _cyl(th=0.5)
    x = np.array([0.0, 0.0, 0.3e-3])
    l0, a = O.pair_areas_mode(tr, x, C, 0.0, 50e6, O.MODE_TRAPEZOID, 1)
    l1, b = O.pair_areas(tr, x, C, 0.0, 50e6)
    assert l0 == l1
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-13 * _tot_cyl(tr))


@pytest.mark.parametrize("seed", range(4))
def test_trapezoid_conserves_total_area(seed):
    rng = np.random.default_rng(40 + seed)
    tr = _cyl(th=rng.uniform(0.1, 0.6))
    x = rng.uniform(-2e-3, 2e-3, 3)
    l0, a = O.pair_areas_mode(tr, x, C, 0.0, 50e6, O.MODE_TRAPEZOID, 1)
    assert a.sum() == pytest.approx(_tot_cyl(tr), rel=1e-12)


def test_trapezoid_error_is_second_order_in_the_aperture():
    """Halving the angular half-aperture (and the arc of every level curve with
    it) divides the error of the trapezoidal I_l by ~4.  The voxel lies beyond
    the axial end of the surface, so Psi(u, r) >= v_min > 0 is smooth on every
    arc; where an arc reaches Psi = 0 (the fold line v = 0) Psi has a square-root
    profile and the chord's error does not shrink with the arc."""
    x = np.array([1.5e-3, 0.0, 2.0e-3])
    errs = []
    for th in (0.2, 0.1, 0.05):
        tr = _cyl(th=th, R=8e-3)
        _, a = O.pair_areas_mode(tr, x, C, 0.0, 50e6, O.MODE_TRAPEZOID, 1)
        _, b = O.pair_areas(tr, x, C, 0.0, 50e6)
        errs.append(np.abs(a - b).sum() / np.abs(b).sum())
    assert errs[0] > 0
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.0 < e0 / e1 < 5.0, errs


def test_trapezoid_leaves_planar_transducers_exact():
    p = P.small_case(P.PLANAR, n=4, K=2, L=160)
    assert rel_l2(O.forward(p, mode=O.MODE_TRAPEZOID), O.forward(p)) < 1e-14


def test_trapezoid_operator_is_adjoint():
    p = P.small_case(P.CYLINDER, n=5, K=3, U=2, L=300, B=2)
    s = O.forward(p, mode=O.MODE_TRAPEZOID)
    z = O.adjoint(p, mode=O.MODE_TRAPEZOID)
    lhs, rhs = np.sum(s * p.y), np.sum(z * p.coef)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(s) * np.linalg.norm(p.y)
    assert rel_l2(s, O.forward(p)) > 0
