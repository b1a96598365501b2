"""High-precision pins of the oracle's cylinder shell areas at degenerate
positions: a voxel on the focal line (rho = 0), one in the plane of an axial
end (a folded v-interval touching 0), one on the back of the aperture (the
folded u-interval reaching pi) and a generic one.

The reference is the definition of the shell area, not Alg. 4: R times the
integral over the axial coordinate v of the angular measure of the surface
points at distance in [r0, r1), evaluated by mpmath at 30 digits with the
integrand's kinks as breakpoints.  The oracle's FP64 areas must agree to
1e-12 of the surface area (the scipy version of this pin allows 1e-9)."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O
import pat_inputs as P

C = P.SOUND_SPEED


def _cyl_area_mp(tr, x, r0, r1):
    mp.mp.dps = 30
    e1, e2, c0 = [np.asarray(tr[a:a + 3]) for a in (4, 7, 1)]
    n3 = np.cross(e1, e2)
    d = [mp.mpf(float(v)) for v in (np.asarray(x) - c0)]
    x1 = sum(d[i] * mp.mpf(float(e2[i])) for i in range(3))
    x2 = sum(d[i] * mp.mpf(float(n3[i])) for i in range(3))
    x3 = sum(d[i] * mp.mpf(float(e1[i])) for i in range(3))
    R, th, Lz = mp.mpf(tr[12]), mp.mpf(tr[13]), mp.mpf(tr[14])
    rho = mp.sqrt(x1 * x1 + x2 * x2)
    thi = mp.atan2(x2, x1) if rho > 0 else mp.mpf(0)
    r0, r1 = mp.mpf(r0), mp.mpf(r1)

    def meas(rr, v):
        q = rr * rr - v * v
        if rho == 0:
            return 2 * th if R * R < q else mp.mpf(0)
        cval = (rho * rho + R * R - q) / (2 * R * rho)
        if cval >= 1:
            return mp.mpf(0)
        if cval <= -1:
            return 2 * th
        a = mp.acos(cval)
        tot = mp.mpf(0)
        for k in (-1, 0, 1):
            lo2, hi2 = thi - a + 2 * mp.pi * k, thi + a + 2 * mp.pi * k
            tot += max(mp.mpf(0), min(hi2, th) - max(lo2, -th))
        return tot

    lo, hi = -Lz - x3, Lz - x3
    pts = [mp.mpf(0)]
    for rr in (r0, r1):
        for phi in (th - thi, -th - thi, mp.mpf(0), mp.pi):
            q = rr * rr - (rho * rho + R * R - 2 * R * rho * mp.cos(phi))
            if q > 0:
                pts += [mp.sqrt(q), -mp.sqrt(q)]
    pts = sorted(set(p for p in pts if lo < p < hi))
    nodes = [lo] + pts + [hi]
    return R * mp.quad(lambda v: meas(r1, v) - meas(r0, v), nodes)


def _tr():
    g = 1.0 + math.sqrt(2.0) * 1e-3
    return P.cylinder([0, 0, 0], [0, 0, 1], [1, 0, 0], 4e-3 * g, 0.4, 0.3e-3)


CASES = {
    "focal_line": [0.0, 0.0, 0.1e-3],
    "axial_end": [0.2e-3, -0.1e-3, -0.3e-3],
    "back_of_aperture": [-0.5e-3, 0.0, 0.1e-3],
    "generic": [0.31e-3, -0.17e-3, 0.05e-3],
}


@pytest.mark.parametrize("case", list(CASES))
def test_cylinder_areas_at_degenerate_positions(case):
    tr = _tr()
    x = np.array(CASES[case])
    fs = 200e6
    l0, a = O.pair_areas(tr, x, C, 0.0, fs)
    dr = C / fs
    tot = 2 * tr[13] * tr[12] * 2 * tr[14]
    assert len(a) > 0
    step = max(1, len(a) // 6)
    for j in list(range(0, len(a), step)) + [len(a) - 1]:
        r0, r1 = (l0 + j - 1) * dr, (l0 + j) * dr
        ref = float(_cyl_area_mp(tr, x, r0, r1))
        assert a[j] == pytest.approx(ref, abs=1e-12 * tot), (case, j)
    assert a.sum() == pytest.approx(tot, rel=1e-13)
