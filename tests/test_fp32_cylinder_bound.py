"""Why the cylinder's shell areas are evaluated in FP64: a measurement.

Alg. 4 obtains each shell area as a difference of edge quantities (Eq.
area_D_l_xi): the arc-integral I_l of Eq. cyl_Il at consecutive edges and the
end-point angle steps, whose difference is ~B/25 .. B/1000 of the terms (B the
bins a quadrant spans).  This test evaluates that difference with FP32 edge
arithmetic in its most favourable form: every per-edge input (the half-angle
sines of the end points, the amplitude of Legendre's addition theorem with its
cosine and Delta, the parameter nu, K = r^2 - (R - rho)^2 and the exact angle
steps) is computed in FP64 and rounded once to FP32, and only Carlson's E, the
addition-theorem combination and the area difference run in FP32 -- any FP32
evaluation of the edges carries at least these roundings.  The FP64 run of the
same code is checked against the oracle first.

On the 128^3 x 256-cylinder workload (a 30 000-voxel sample of transducer 0
here) the FP32 areas are off by ~2e-4 RMS per bin and the signal of that
sample by ~4e-5 relative L2; over the whole volume (run this file as a script:
all 2 045 585 nonzero voxels, transducers 0 and 131) the per-bin errors average
in f to ~2e-6 but the zero-mean system kernel's cancellation lifts the signal
error to 1.3e-4 .. 1.4e-4, 13x over the 1e-5 target.  The FP32 unpacked vector
rate is twice the FP64 rate on gfx950, so an FP32 edge path would have paid;
it cannot hold the accuracy.
"""
import sys

import numpy as np

import oracle as O
import pat_inputs as P
from conftest import rel_l2


def carlson_e(s, c, dl, nu, dt):
    """E(sigma, nu) = s R_F(c^2, dl^2, 1) - nu/3 s^3 R_D(c^2, dl^2, 1) (DLMF
    19.25.9), Carlson's duplication and the series of DLMF 19.36.1-2, every
    operation in the type ``dt``."""
    s, c, dl, nu = (np.asarray(v, dtype=dt) for v in (s, c, dl, nu))
    x, y, z = c * c, dl * dl, np.ones_like(c)
    sum_d, p4 = np.zeros_like(c), np.ones_like(c)
    three, five = dt(3), dt(5)
    for it in range(12):
        a = (x + y + three * z) / five
        dev = np.maximum(np.abs(a - x), np.maximum(np.abs(a - y), np.abs(a - z)))
        if it > 0 and np.all(dev * dt(35) < a):
            break
        sx, sy, sz = np.sqrt(x), np.sqrt(y), np.sqrt(z)
        lam = sx * sy + sx * sz + sy * sz
        sum_d = sum_d + p4 / (sz * (z + lam))
        p4 = p4 / dt(4)
        x, y, z = (x + lam) / dt(4), (y + lam) / dt(4), (z + lam) / dt(4)
    af = (x + y + z) / three
    X, Y = (af - x) / af, (af - y) / af
    Z = -X - Y
    e2, e3 = X * Y - Z * Z, X * Y * Z
    rf = (dt(1) - e2 / dt(10) + e3 / dt(14) + e2 * e2 / dt(24) - three * e2 * e3 / dt(44)
          - dt(5) * e2 * e2 * e2 / dt(208) + three * e3 * e3 / dt(104) + e2 * e2 * e3 / dt(16)) / np.sqrt(af)
    ad = (x + y + three * z) / five
    X, Y = (ad - x) / ad, (ad - y) / ad
    Z = -(X + Y) / three
    xy, z2 = X * Y, Z * Z
    d2, d3 = xy - dt(6) * z2, (three * xy - dt(8) * z2) * Z
    d4, d5 = three * (xy - z2) * z2, xy * z2 * Z
    ser = (dt(1) - three * d2 / dt(14) + d3 / dt(6) + dt(9) * d2 * d2 / dt(88) - three * d4 / dt(22)
           - dt(9) * d2 * d3 / dt(52) + three * d5 / dt(26))
    rd = three * sum_d + p4 * ser / (ad * np.sqrt(ad))
    return s * rf - nu / three * s * s * s * rd


def _quadrants(tr, X):
    """Reflected quadrants (Eq. folded_intervals, Eq. uvminmax), unmerged:
    rows (pair, a, b, c, d, rho)."""
    c0, e1, e2 = tr[1:4], tr[4:7], tr[7:10]
    n3 = np.cross(e1, e2)
    th, lz = tr[13], tr[14]
    d = X - c0
    x1, x2, x3 = d @ e2, d @ n3, d @ e1
    rho, thi = np.hypot(x1, x2), np.arctan2(x2, x1)

    def wrap(u):
        return np.where(u <= -np.pi, u + 2 * np.pi, np.where(u > np.pi, u - 2 * np.pi, u))
    u1, u2 = wrap(-th - thi), wrap(th - thi)
    c1 = (u1 < 0) & (0 < u2)
    c2 = ~c1 & (u2 < u1)
    c3 = ~c1 & ~c2 & (0 <= u1)
    us = [(np.where(c1, 0.0, np.where(c2 | c3, u1, -u2)), np.where(c1, -u1, np.where(c2, np.pi, np.where(c3, u2, -u1)))),
          (np.where(c1 | c2, np.where(c1, 0.0, -u2), 0.0), np.where(c1, u2, np.where(c2, np.pi, 0.0)))]
    v1, v2 = -lz - x3, lz - x3
    vs = [(np.maximum(v1, 0), np.maximum(v2, 0)), (np.maximum(-v2, 0), np.maximum(-v1, 0))]
    rows = []
    for a, b in us:
        for c, dd in vs:
            i = np.nonzero((b > a) & (dd > c))[0]
            rows.append(np.stack([i, a[i], b[i], c[i], dd[i], rho[i]], axis=1))
    return np.concatenate(rows)


def shell_areas(tr, X, c_s, t0, ufs):
    """Areas of every (quadrant, bin) of the voxels X on cylinder ``tr`` by Alg. 4,
    the edge differences in FP64 and, from the same FP64 edge inputs rounded
    once, in FP32.  Returns (pair, bin, area64, area32)."""
    R = tr[12]
    q = _quadrants(tr, X)
    pair, a, b, c, d, rho = q.T
    dm, dp = R - rho, R + rho

    def psi(u, rh):
        return (R - rh) ** 2 + 4 * R * rh * np.sin(0.5 * u) ** 2
    l0 = np.floor((np.sqrt(psi(a, rho) + c * c) / c_s - t0) * ufs).astype(np.int64) + 1
    l1 = np.ceil((np.sqrt(psi(b, rho) + d * d) / c_s - t0) * ufs).astype(np.int64)
    n = l1 - l0 + 1
    qi = np.repeat(np.arange(len(q)), n)
    off = np.arange(qi.size) - np.repeat(np.cumsum(n) - n, n)
    binl = l0[qi] + off
    r2 = (c_s * (t0 + binl / ufs)) ** 2
    A, B, C, D, DM, DP, RH = a[qi], b[qi], c[qi], d[qi], dm[qi], dp[qi], rho[qi]
    pa, pb = psi(A, RH), psi(B, RH)

    def half_angle(qv):   # clamped inverse of the level curve on a line (Eq. alphabeta), halved
        inner = np.arctan2(np.sqrt(np.maximum(qv - DM * DM, 0)), np.sqrt(np.maximum(DP * DP - qv, 0)))
        return np.where(qv <= pa, 0.5 * A, np.where(qv >= pb, 0.5 * B, inner))
    ha, hb = half_angle(r2 - D * D), half_angle(r2 - C * C)
    K = r2 - DM * DM
    act = (hb > ha) & (K > 0)
    K = np.where(act, K, 1.0)
    nu = 4 * R * RH / K
    sa, sb, ca, cb = np.sin(ha), np.sin(hb), np.cos(ha), np.cos(hb)
    da, db = np.sqrt(np.maximum(1 - nu * sa * sa, 0)), np.sqrt(np.maximum(1 - nu * sb * sb, 0))
    # Legendre's addition theorem: F(sigma) = F(beta/2) - F(alpha/2), then
    # E(beta/2) - E(alpha/2) = E(sigma) - nu sin(alpha/2) sin(beta/2) sin(sigma)
    den = cb * cb + (sb * da) ** 2
    ss = np.where(act, (sb * da * ca - sa * cb * db) / den, 0.0)
    cs = np.where(act, (cb * ca + sb * sa * da * db) / den, 1.0)
    ds = np.where(act, (nu * sb * sa * cb * ca + da * db) / den, 1.0)
    first = off == 0

    def prev(v, start):
        return np.where(first, start, np.roll(v, 1))
    dal, dbe = 2 * (ha - prev(ha, 0.5 * A)), 2 * (hb - prev(hb, 0.5 * A))
    out = []
    for dt in (np.float64, np.float32):
        e = carlson_e(ss.astype(dt), cs.astype(dt), ds.astype(dt), nu.astype(dt), dt)
        i_l = np.where(act, dt(2) * np.sqrt(K.astype(dt)) * (e - nu.astype(dt) * sa.astype(dt) * sb.astype(dt)
                                                             * ss.astype(dt)), dt(0))
        area = dt(R) * (dal.astype(dt) * D.astype(dt) + (i_l - prev(i_l, dt(0))) - dbe.astype(dt) * C.astype(dt))
        out.append(area.astype(np.float64))
    return pair[qi].astype(np.int64), binl, out[0], out[1]


def signal_errors(p, h, k, voxels):
    """FP32 against FP64: per-bin relative RMS over bins above 1e-3 of the
    largest, f and signal relative L2, and the FP64 run against the oracle."""
    tr = p.tr.packed[k]
    ufs = p.U * p.fs
    X = p.grid.coords()[voxels]
    pair, binl, a64, a32 = shell_areas(tr, X, p.sound_speed, p.t0, ufs)
    worst = 0.0
    for j in range(0, len(voxels), max(1, len(voxels) // 8)):
        l0, ref = O.pair_areas(tr, X[j], p.sound_speed, p.t0, ufs)
        m = pair == j
        got = np.zeros(len(ref))
        np.add.at(got, binl[m] - l0, a64[m])
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(ref)))
    key = pair * (binl.max() - binl.min() + 1) + (binl - binl.min())
    _, inv = np.unique(key, return_inverse=True)
    b64, b32 = np.bincount(inv, a64), np.bincount(inv, a32)
    big = b64 > 1e-3 * b64.max()
    per_bin = float(np.sqrt(np.mean(((b32 - b64)[big] / b64[big]) ** 2)))
    m0 = binl.min()
    tau = p.t0 + (np.arange(m0, binl.max() + 1) - 0.5) / ufs
    w = p.coef[0][voxels][pair]
    f64 = np.bincount(binl - m0, w * a64) / (p.sound_speed * tau)
    f32 = np.bincount(binl - m0, w * a32) / (p.sound_speed * tau)
    return worst, per_bin, rel_l2(f32, f64), rel_l2(np.convolve(h, f32), np.convolve(h, f64))


def test_fp32_carlson_matches_scipy_to_fp32_rounding():
    from scipy.special import elliprd, elliprf
    rng = np.random.default_rng(0)
    nu = rng.uniform(0, 5, 2000)
    s = np.minimum(rng.uniform(0, 1, 2000), 0.999 / np.sqrt(np.maximum(nu, 1)))
    c, dl = np.sqrt(1 - s * s), np.sqrt(1 - nu * s * s)
    ref = s * elliprf(c * c, dl * dl, 1) - nu / 3 * s ** 3 * elliprd(c * c, dl * dl, 1)
    assert np.max(np.abs(carlson_e(s, c, dl, nu, np.float64) - ref)) < 1e-13
    e32 = carlson_e(s, c, dl, nu, np.float32).astype(np.float64)
    assert np.max(np.abs(e32 - ref) / np.maximum(np.abs(ref), 1e-3)) < 2e-6


def test_fp32_cylinder_edges_miss_the_target():
    p = P.cyl256_128c()
    h, _ = O.kernel_of(p)
    nz = np.nonzero(p.coef[0])[0]
    voxels = np.sort(np.random.default_rng(1).choice(nz, size=30000, replace=False))
    worst, per_bin, ef, es = signal_errors(p, h, 0, voxels)
    print(f"emulation FP64 vs oracle {worst:.2e}; FP32 per-bin RMS {per_bin:.2e}, f {ef:.2e}, signal {es:.2e}")
    assert worst < 1e-9                      # the FP64 run of the emulation is Alg. 4
    assert per_bin > 5e-5 and es > 1e-5      # FP32 edges: ~2e-4 per bin, ~4e-5 on the sample's signal


if __name__ == "__main__":
    # the whole volume: every nonzero voxel of the workload, in chunks
    p = P.cyl256_128c()
    h, _ = O.kernel_of(p)
    nz = np.nonzero(p.coef[0])[0]
    for k in [int(a) for a in sys.argv[1:]] or [0, 131]:
        acc = {}
        tr = p.tr.packed[k]
        ufs = p.U * p.fs
        parts = []
        for s0 in range(0, len(nz), 60000):
            v = nz[s0:s0 + 60000]
            pair, binl, a64, a32 = shell_areas(tr, p.grid.coords()[v], p.sound_speed, p.t0, ufs)
            w = p.coef[0][v][pair]
            parts.append((binl, w * a64, w * a32))
        m0 = min(b.min() for b, _, _ in parts)
        m1 = max(b.max() for b, _, _ in parts)
        f64 = sum(np.bincount(b - m0, x, minlength=m1 - m0 + 1) for b, x, _ in parts)
        f32 = sum(np.bincount(b - m0, y, minlength=m1 - m0 + 1) for b, _, y in parts)
        tau = p.t0 + (np.arange(m0, m1 + 1) - 0.5) / ufs
        f64, f32 = f64 / (p.sound_speed * tau), f32 / (p.sound_speed * tau)
        print(f"transducer {k}, all {len(nz)} nonzero voxels: f rel L2 {rel_l2(f32, f64):.2e}, "
              f"signal rel L2 {rel_l2(np.convolve(h, f32), np.convolve(h, f64)):.2e}", flush=True)
