"""The precision of the cylinder kernels' elliptic integral E(sigma | nu) at
their two duplication stops, on the CPU.

`ellip_e_model` restates, in numpy, the steps the kernels take for
E = s R_F(c^2, D^2, 1) - nu s^3 R_D(c^2, D^2, 1) / 3 (DLMF 19.25.9): Carlson's
duplication on 4^n-scaled iterates with its first step peeled, stopped once
stop x max |A - x_i| < A, then the series of DLMF 19.36.1-2 through degree 7,
in FP64 (the FP64 kernels, stop 35) or with the terms beyond the leading 1 in
FP32 (the FP32-I/O kernels, stop 12).  The reference is mpmath's incomplete
integral at 30 digits, over amplitudes from 1e-3 to 1.55 rad and parameters up
to nu sin^2 sigma = 0.99999 (the near-tangent edges, where Delta -> 0).  The
bars are what the kernels' comments and the design notes claim: ~1e-13 for the
FP64 kernels, and for the FP32-I/O kernels ~5e-10, dominated by the FP32 series
terms, which the signals' FP32 rounding (6e-8) covers even after the ~10^2-10^3
cancellation of the edge differences.  Not a parity test: the kernels' own
output is checked against the oracle by the GPU tests."""
import math

import mpmath as mp
import numpy as np
import pytest


def ellip_e_model(s, c, dl, nu, stop, f32_series):
    s, c, dl, nu = (np.asarray(v, dtype=np.float64) for v in (s, c, dl, nu))
    tiny = 1e-30
    x = c * c + tiny
    y = dl * dl + tiny
    z = np.ones_like(x)
    sx, sy, sz = np.abs(c), dl.copy(), np.ones_like(x)
    AF = (x + y + z) / 3.0
    AD = (x + y + 3.0 * z) * 0.2
    thr = stop * np.maximum(z - AF, AD - np.minimum(x, y))
    p2 = np.ones_like(x)
    sumD = np.zeros_like(x)
    act = thr >= AF
    # the first step, where z = sqrt(z) = 1
    lam = sx * sy + sx + sy
    z = np.where(act, z + lam, z)
    sumD = np.where(act, 1.0 / z, sumD)
    x, y, AF = (np.where(act, v + lam, v) for v in (x, y, AF))
    p2 = np.where(act, 2.0, p2)
    sx, sy, sz = (np.where(act, np.sqrt(v), w) for v, w in ((x, sx), (y, sy), (z, sz)))
    for _ in range(1, 12):
        act = act & (thr >= AF)
        if not act.any():
            break
        lam = sx * sy + sx * sz + sy * sz
        sumD = np.where(act, sumD + p2 / (sz * (z + lam)), sumD)
        x, y, z, AF = (np.where(act, v + lam, v) for v in (x, y, z, AF))
        p2 = np.where(act, 2.0 * p2, p2)
        sx, sy, sz = (np.where(act, np.sqrt(v), w) for v, w in ((x, sx), (y, sy), (z, sz)))
    AD = (x + y + 3.0 * z) * 0.2
    rAF, rAD = 1.0 / np.sqrt(AF), 1.0 / np.sqrt(AD)
    X, Y = (AF - x) * rAF * rAF, (AF - y) * rAF * rAF
    Xd, Yd = (AD - x) * rAD * rAD, (AD - y) * rAD * rAD
    T = np.float32 if f32_series else np.float64
    X, Y, Xd, Yd = (v.astype(T) for v in (X, Y, Xd, Yd))
    c_ = [T(v) for v in (-5.0 / 208, 1.0 / 24, 0.1, 1.0 / 16, -3.0 / 44, 3.0 / 104, 1.0 / 14)]
    Z = -X - Y
    E2, E3 = X * Y - Z * Z, X * Y * Z
    df = E2 * (E2 * (E2 * c_[0] + c_[1]) - c_[2]) + E3 * (E2 * (E2 * c_[3] + c_[4]) + (E3 * c_[5] + c_[6]))
    rf = (1.0 + df.astype(np.float64)) * rAF * p2
    Zd = -(Xd + Yd) * T(1.0 / 3.0)
    XY, Z2 = Xd * Yd, Zd * Zd
    D2, D3 = XY - T(6.0) * Z2, (T(3.0) * XY - T(8.0) * Z2) * Zd
    D4, D5 = T(3.0) * (XY - Z2) * Z2, XY * Z2 * Zd
    t2 = D3 * T(45.0 / 272) + (D2 * T(-1.0 / 16) + T(9.0 / 88))
    t2 = D2 * t2 + (D3 * T(-9.0 / 52) + (D4 * T(3.0 / 20) + (D5 * T(-9.0 / 68) + T(-3.0 / 14))))
    t3 = D3 * T(3.0 / 40) + (D4 * T(-9.0 / 68) + T(1.0 / 6))
    dd = D2 * t2 + (D3 * t3 + (D4 * T(-3.0 / 22) + D5 * T(3.0 / 26)))
    rd = p2 * (1.0 + dd.astype(np.float64)) * rAD * rAD * rAD + 3.0 * sumD
    return s * (rf - nu / 3.0 * s * s * rd)


def _grid():
    mp.mp.dps = 30
    rows = []
    for sg in (1e-3, 0.01, 0.05, 0.1, 0.2, 0.4, 0.6, 0.8, 1.0, 1.2, 1.4, 1.55):
        for q in (0.0, 0.1, 0.3, 0.6, 0.9, 0.99, 0.999, 0.99999):
            s = math.sin(sg)
            nu = q / (s * s)
            ref = float(mp.ellipe(mp.asin(mp.mpf(s)), mp.mpf(nu)))
            rows.append((s, math.cos(sg), math.sqrt(1.0 - nu * s * s), nu, ref))
    return np.array(rows).T


@pytest.mark.parametrize("stop,f32_series,bar", [(35.0, False, 1e-13), (12.0, True, 1e-9)],
                         ids=["fp64_kernels", "fp32_io_kernels"])
def test_duplication_stop_precision(stop, f32_series, bar):
    s, c, dl, nu, ref = _grid()
    e = ellip_e_model(s, c, dl, nu, stop, f32_series)
    rel = np.abs(e - ref) / np.abs(ref)
    print(f"stop {stop:g}, {'FP32' if f32_series else 'FP64'} series: max relative error {rel.max():.3e}, "
          f"median {np.median(rel):.3e}")
    assert rel.max() < bar


def test_looser_stop_costs_less_than_the_fp32_series():
    """At the FP32-I/O stop the series' truncation alone (FP64 terms) stays far
    below the FP32 terms' rounding, so a tighter stop would buy nothing there."""
    s, c, dl, nu, ref = _grid()
    trunc = np.abs(ellip_e_model(s, c, dl, nu, 12.0, False) - ref) / np.abs(ref)
    both = np.abs(ellip_e_model(s, c, dl, nu, 12.0, True) - ref) / np.abs(ref)
    print(f"stop 12: truncation {trunc.max():.3e}, with the FP32 series {both.max():.3e}")
    assert trunc.max() < 0.1 * both.max()
