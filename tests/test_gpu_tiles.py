"""The (transducer, time tile) forward against the FP64 oracle, element by
element through the C ABI, and against the cube forward.

In this forward one work-group owns a tile of consecutive area shells of one
transducer's fine-bin vector f_k (Eq. ui_area) and stores it, with no fill and
no atomics; it finds its voxels by scanning the bricks whose bounding-sphere
window meets the tile and clips every pair's sweep to the tile.  The cases
cover tiles narrower than one pair's shell range (32 shells), the automatic
width, a ragged last tile, one to six volumes (the kernels for 1, 2, 4 and 8
right-hand sides), the coarse area grid (a tile of shells is step x tile fine
bins), both shape groups in one geometry, the trapezoidal and lookup-table
cylinder I_l, and the refusal of the quadrature mode and of invalid widths.

Bars: those of the cube forward against the oracle (FP32 1e-5 relative L2
and the per-row bound ROW_TAU, FP64 1e-11).  Against the cube forward: each
area is evaluated as in the cube forward (a planar quadrant is walked from its
first bin whatever the tile, a cylinder edge on its own) and the two forwards
sum the same FP64 terms in other groupings, so FP64 rows agree to 1e-13 of
their largest sample and FP32 rows to one unit in the last place away from
zero crossings (the determinism tests' bar for two runs of one forward; at
full size, one unit in the last place of the row's largest sample).
"""
import numpy as np
import pytest
import torch

import oracle as O
import pat_inputs as P
from conftest import ROW_TAU, ROW_TAU_FULL, fp32_repeat_ok, rel_l2, row_ratio

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-11}
DT = {"fp32": torch.float32, "fp64": torch.float64}
OMODE = {"closed": O.MODE_SURFACE, "trapezoid": O.MODE_TRAPEZOID, "lut": O.MODE_LUT}


def forward_gpu(prob, mode, prec, step, tiles):
    from paper_2609_29253_amd.operator import PatOperator
    B = prob.coef.shape[0]
    op = PatOperator.from_problem(prob, mode=mode, precision=prec, max_batch=B, area_step=step, time_tiles=tiles)
    width = op.query(9)
    s = op.forward(torch.tensor(prob.coef, dtype=DT[prec], device="cuda"))
    torch.cuda.synchronize()
    out = s.cpu().numpy()
    op.close()
    return out, width


def cube_agreement(prec, s_tile, s_cube):
    """(measure, bar): FP64, the largest per-row difference over the row's
    largest sample; FP32, the largest ulp distance away from zero crossings."""
    if prec == "fp64":
        return row_ratio(s_tile, s_cube), 1e-13
    return fp32_repeat_ok(s_tile, s_cube), 1


CASES = [
    # shape, U, step, B, n, K, L, mode, tile (0 = automatic)
    (P.CYLINDER, 1, 1, 1, 13, 5, 260, "closed", 32),
    (P.CYLINDER, 1, 1, 2, 13, 5, 260, "closed", 0),
    (P.CYLINDER, 4, 2, 3, 9, 3, 260, "closed", 64),
    (P.CYLINDER, 2, 1, 6, 7, 3, 260, "closed", 32),
    (P.PLANAR, 1, 1, 1, 13, 5, 200, "closed", 32),
    (P.PLANAR, 3, 3, 2, 9, 4, 200, "closed", 0),
    (P.PLANAR, 2, 1, 5, 7, 3, 200, "closed", 128),
    (P.CYLINDER, 2, 1, 2, 9, 4, 260, "trapezoid", 32),
    (P.CYLINDER, 1, 1, 1, 11, 4, 260, "lut", 64),
]


def _id(c):
    return f"{'pl' if c[0] == 0 else 'cy'}_U{c[1]}_step{c[2]}_B{c[3]}_n{c[4]}_{c[7]}_t{c[8]}"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("case", CASES, ids=_id)
def test_tiles_against_oracle_and_cubes(gpu, case, prec):
    shape, U, step, B, n, K, L, mode, tile = case
    p = P.small_case(shape, n=n, K=K, U=U, B=B, L=L, seed=4)
    print(f"case {p.name} U={U} step={step} B={B} {mode} tile={tile} {prec}", flush=True)
    s_ref = O.forward(p, mode=OMODE[mode], step=step)
    s, width = forward_gpu(p, mode, prec, step, tile)
    assert width == (tile if tile else width) and 32 <= width <= 512
    s_cube, off = forward_gpu(p, mode, prec, step, None)
    assert off == 0
    e, r = rel_l2(s, s_ref), row_ratio(s, s_ref)
    agree, bar = cube_agreement(prec, s, s_cube)
    print(f"  tile {width:.0f}: rel L2 {e:.3e}, worst row {r:.3e}; against the cube forward "
          f"{agree:.3g} (bar {bar:g})", flush=True)
    assert np.linalg.norm(s_ref) > 0
    assert e < TOL[prec] and r <= ROW_TAU[prec]
    assert agree <= bar


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("tile", [32, 0])
def test_tiles_mixed_shapes(gpu, prec, tile):
    """Planar and cylindrical transducers in one geometry: two shape groups,
    each with its own sorted work items."""
    p = P.mixed_case(n=13, K_planar=3, K_cyl=3, L=300, seed=2, B=2)
    s_ref = O.forward(p)
    s, width = forward_gpu(p, "closed", prec, 1, tile)
    s_cube, _ = forward_gpu(p, "closed", prec, 1, None)
    e, r = rel_l2(s, s_ref), row_ratio(s, s_ref)
    agree, bar = cube_agreement(prec, s, s_cube)
    print(f"mixed tile {width:.0f} {prec}: rel L2 {e:.3e}, worst row {r:.3e}, against cubes {agree:.3g} "
          f"(bar {bar:g})", flush=True)
    assert e < TOL[prec] and r <= ROW_TAU[prec]
    assert agree <= bar


def test_tiles_zero_input_and_refusals(gpu):
    """A zero volume gives an exactly zero signal (every fine bin is stored by
    its tile, none is left from an earlier call); the quadrature mode and
    widths outside 32..512 or not powers of two are refused."""
    from paper_2609_29253_amd import _lib as L
    from paper_2609_29253_amd.operator import PatOperator
    p = P.small_case(P.CYLINDER, n=9, K=3, L=200, seed=5, B=1)
    op = PatOperator.from_problem(p, mode="closed", precision="fp32", max_batch=1, time_tiles=32)
    c = torch.tensor(p.coef, dtype=torch.float32, device="cuda")
    s1 = op.forward(c)
    s0 = op.forward(torch.zeros_like(c))
    s2 = op.forward(c)
    torch.cuda.synchronize()
    assert float(s1.abs().max()) > 0
    assert torch.count_nonzero(s0).item() == 0
    assert fp32_repeat_ok(s1.cpu().numpy(), s2.cpu().numpy()) <= 1
    op.close()
    with pytest.raises(RuntimeError, match="time-tile"):
        PatOperator.from_problem(p, mode="quadrature", precision="fp32", max_batch=1, time_tiles=0)
    for bad in (16, 48, 1024):
        with pytest.raises(ValueError):
            PatOperator.from_problem(p, mode="closed", precision="fp32", max_batch=1, time_tiles=bad)
    assert L.PAT_FLAG_TIME_TILES == 1


def row_ratios(got, ref):
    """Per row max |got - ref| / max |ref| (rows: the last axis)."""
    g = np.asarray(got, dtype=np.float64).reshape(-1, got.shape[-1])
    r = np.asarray(ref, dtype=np.float64).reshape(-1, ref.shape[-1])
    return np.max(np.abs(g - r), axis=1) / np.maximum(np.max(np.abs(r), axis=1), 1e-300)


@pytest.mark.slow
@pytest.mark.parametrize("name,ks", [("cyl256_128c", [0, 131]), ("planar512_256c", [0, 301])])
def test_tiles_full_size(gpu, name, ks):
    """The benchmark's workloads with the automatic width, FP32 I/O.  Every
    row against the cube forward; the oracle on two fixed transducers and on
    the row where the two forwards differ most, over every voxel, where both
    forwards must meet the per-row bound.  Rows agree to one FP32 unit in the
    last place of the row's largest sample: the two forwards sum the same terms
    in other groupings (a fine bin sums ~3e4 at this size), and the cylinder
    angle steps follow a wave-wide choice of method (each exact to ~1e-13) over
    lanes that differ between the two."""
    p = {"cyl256_128c": P.cyl256_128c, "planar512_256c": P.planar512_256c}[name]()
    s, width = forward_gpu(p, "closed", "fp32", 1, 0)
    s_cube, _ = forward_gpu(p, "closed", "fp32", 1, None)
    d = row_ratios(s, s_cube)
    worst = int(np.argmax(d))
    check = sorted(set(ks) | {worst})
    s_ref = O.forward(p, ksub=np.asarray(check, dtype=np.int32))
    got, cube = s[:, check, :], s_cube[:, check, :]
    e, r = rel_l2(got, s_ref), row_ratio(got, s_ref)
    eb, rb = rel_l2(cube, s_ref), row_ratio(cube, s_ref)
    bar = 2.0 ** -23
    print(f"[{name}] tile {width:.0f}: rows against the cube forward: largest difference {d.max():.3e} of the "
          f"row maximum (transducer {worst}, bar {bar:.3g}), median {np.median(d):.3e}; oracle on transducers "
          f"{check}: tile rel L2 {e:.3e}, worst row {r:.3e}; cube rel L2 {eb:.3e}, worst row {rb:.3e}",
          flush=True)
    assert e < TOL["fp32"] and r <= ROW_TAU_FULL["fp32"]
    assert eb < TOL["fp32"] and rb <= ROW_TAU_FULL["fp32"]
    assert d.max() <= bar
