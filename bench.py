#!/usr/bin/env python3
"""Throughput of the matrix-free photoacoustic operator A and its adjoint A^T.

One step = one application of A followed by one application of A^T to the
whole synthetic input (all volumes of the workload), through the C ABI.
Prints one JSON line (rank 0) with the A+A^T voxel x transducer pair rate,
the roofline of the dominant kernel and the FP64 oracle's rate on the host
cores for a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload cyl256_128c] [--no-variants] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A+Aᵀ voxel×transducer pairs/s, closed-form FP32 vs quadrature/FP64 at rel err"

# Algorithmic FLOPs of the dominant kernel per area evaluation (one quadrant of
# one voxel-transducer pair in one fine bin) are read from its own instruction
# counters, committed under profiles/ as "flops-json" lines: the FP64 and FP32
# FMA (2 FLOP), MUL, ADD and transcendental (1 FLOP each) wave instructions of
# one launch, times 64 lanes, times the measured lane activity
# SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU) (the operations the active
# lanes executed), over that launch's area evaluations.
PEAKS = {"f32": 157.3e12, "f64": 78.6e12}


def kernel_source_hash():
    """Hash of the device sources with comments and blank space removed: a
    change of the kernels' code changes it, a change of their comments does not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("area.h", "kernels.hip", "kernels.h", "patop_internal.h"):
        with open(os.path.join(ROOT, "paper_2609_29253_amd", "csrc", f)) as fh:
            txt = fh.read()
        txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", " ", txt)
        h.update(" ".join(txt.split()).encode())
    return h.hexdigest()[:16]


def profile_records(kind):
    """The machine-readable "<kind>-json:" lines of the committed summaries."""
    import glob
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        try:
            with open(path) as fh:
                for line in fh:
                    if line.strip().startswith(kind + "-json:"):
                        out.append(json.loads(line.split(":", 1)[1]))
        except (OSError, ValueError):
            pass
    return out


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, calibrated on a plain copy), or None when the kernel sources
    have changed since the counters were taken."""
    for rec in profile_records("traffic"):
        if (rec.get("kernel") == kernel and rec.get("workload") == workload
                and rec.get("source_hash") == kernel_source_hash()):
            return rec["traffic_bytes"]
    return None


def counter_flops(kernel, workload):
    """(FP64 FLOPs, FP32 FLOPs) per area evaluation of ``kernel`` on ``workload``
    from its committed instruction counters, and whether the kernel sources
    still hash to the profiled ones; None without a record."""
    best = None
    for rec in profile_records("flops"):
        if rec.get("kernel") != kernel or rec.get("workload") != workload:
            continue
        c = rec["counters"]
        lam = c["SQ_THREAD_CYCLES_VALU"] / (64.0 * c["SQ_ACTIVE_INST_VALU"])
        per = {}
        for p in ("F64", "F32"):
            ops = (2.0 * c[f"SQ_INSTS_VALU_FMA_{p}"] + c[f"SQ_INSTS_VALU_MUL_{p}"] + c[f"SQ_INSTS_VALU_ADD_{p}"]
                   + c[f"SQ_INSTS_VALU_TRANS_{p}"])
            per[p] = lam * 64.0 * ops / rec["evals_per_launch"]
        cur = rec.get("source_hash") == kernel_source_hash()
        if best is None or cur:
            best = (per["F64"], per["F32"], cur, lam)
    return best


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name):
    import pat_inputs as P
    if name in P.WORKLOADS:
        return P.WORKLOADS[name]()
    raise SystemExit(f"unknown workload {name}")


def time_op(op, coef, y, steps, warmup, torch):
    """Returns (ms per step, ms forward, ms adjoint) averaged over `steps`."""
    for _ in range(warmup):
        op.forward(coef)
        op.adjoint(y)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(st)
        op.forward(coef)
        e1.record(st)
        op.adjoint(y)
        e2.record(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    f = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    a = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    return wall, f, a


def run_tiles(prob, torch, dev, log, steps=3):
    """A/B of the forward's two decompositions on the workload (FP32 I/O,
    closed form): one-wave (4 x 4 x 4 voxel cube, transducer chunk)
    work-groups adding into f with atomics, against 256-thread (transducer,
    time tile) work-groups that own their
    tile of f, at the automatic and at fixed tile widths.  Forward time only
    (the adjoint is the same in both), HIP events on torch's current stream."""
    from paper_2609_29253_amd.operator import PatOperator, build_kernel
    kern = build_kernel(prob.phi_type, prob.kappa, prob.eir, prob.sound_speed, prob.fs, prob.U)
    B = prob.coef.shape[0]
    coef = torch.tensor(prob.coef, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream()
    rows = []
    ref = None
    for tiles in (None, 0, 32, 64, 128, 256, 512):
        op = PatOperator.from_problem(prob, mode="closed", precision="fp32", max_batch=B, kernel=kern,
                                      time_tiles=tiles)
        s = op.forward(coef)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for e0, e1 in ev:
            e0.record(st)
            op.forward(coef)
            e1.record(st)
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in ev) / steps
        out = s.double()
        if ref is None:
            ref = out
        diff = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
        row = {"decomposition": "cubes" if tiles is None else "time tiles",
               "tile_shells": int(op.query(9)), "automatic": tiles == 0, "ms_forward": round(ms, 3),
               "rel_l2_vs_cubes": diff}
        rows.append(row)
        log(f"[bench] tiles {prob.name}: {row}")
        op.close()
    return {"workload": prob.name, "rows": rows}


def run_next(args, prob, kern, B, pairs, torch, dev, log):
    """Approximate variants: time per A + A^T and rel L2 error against the
    oracle's exact method (method error) and its own version of the variant
    (rounding), on bounded samples."""
    import numpy as np
    import oracle as O
    import pat_inputs as P
    from paper_2609_29253_amd.operator import PatOperator, build_kernel

    def rl2(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def timed(p, kern_, mode, step, steps=2):
        if mode == "quadrature":
            step = 1
        op = PatOperator.from_problem(p, mode=mode, precision="fp32", max_batch=B, kernel=kern_, area_step=step)
        coef = torch.tensor(p.coef, dtype=torch.float32, device=dev)
        y = torch.tensor(p.y, dtype=torch.float32, device=dev)
        wall, f_ms, a_ms = time_op(op, coef, y, steps, 1, torch)
        evals = op.query(7)
        s = op.forward(coef).double().cpu().numpy()
        z = op.adjoint(y).double().cpu().numpy()
        op.close()
        return wall, f_ms, a_ms, evals, s, z

    rows = {}
    ks = np.array([0, 131], dtype=np.int32)
    vs = np.linspace(0, prob.N - 1, 512).astype(np.int64)
    h, nf = O.kernel_of(prob)
    shape = 1 if 1 in set(int(v) for v in prob.tr.packed[:, 0]) else 0
    ex = (O.forward(prob, ksub=ks, kernel=(h, nf)), O.adjoint(prob, vsub=vs, kernel=(h, nf)))
    if shape == 1:
        # the two cheaper cylinder I_l: chord of the level curve, lookup tables
        for mode, omode in (("trapezoid", O.MODE_TRAPEZOID), ("lut", O.MODE_LUT)):
            wall, f_ms, a_ms, ev, s, z = timed(prob, kern, mode, 1, max(1, min(3, args.steps)))
            same = (O.forward(prob, ksub=ks, mode=omode, kernel=(h, nf)),
                    O.adjoint(prob, vsub=vs, mode=omode, kernel=(h, nf)))
            rows[f"{mode}_fp32"] = {
                "workload": prob.name, "ms_per_step": round(wall, 3), "ms_forward": round(f_ms, 3),
                "ms_adjoint": round(a_ms, 3), "pairs_per_s": pairs / (wall * 1e-3), "area_evaluations": ev,
                "rel_err_vs_exact_oracle": {"forward": rl2(s[:, ks], ex[0]), "adjoint": rl2(z[:, vs], ex[1])},
                f"rel_err_vs_oracle_{mode}": {"forward": rl2(s[:, ks], same[0]), "adjoint": rl2(z[:, vs], same[1])}}
            log(f"[bench] next {mode}: {rows[f'{mode}_fp32']}")
    # the quadrature refined: error against the exact method and cost as Q grows
    q0 = tuple(prob.quad_n)
    for qn in (32, 64):
        prob.quad_n = (qn, qn)
        wall, f_ms, a_ms, ev, s, z = timed(prob, kern, "quadrature", 1, 1)
        rows[f"quadrature_{qn}x{qn}_fp32"] = {
            "workload": prob.name, "ms_per_step": round(wall, 3), "pairs_per_s": pairs / (wall * 1e-3),
            "rel_err_vs_exact_oracle": {"forward": rl2(s[:, ks], ex[0]), "adjoint": rl2(z[:, vs], ex[1])}}
        log(f"[bench] next quadrature {qn}x{qn}: {rows[f'quadrature_{qn}x{qn}_fp32']}")
    prob.quad_n = q0
    # coarse area grid (Remark 1) at U = 4: every fine bin vs one area per native sample
    p4 = P.cyl256_128c(U=4)
    k4 = build_kernel(p4.phi_type, p4.kappa, p4.eir, p4.sound_speed, p4.fs, p4.U)
    h4, nf4 = O.kernel_of(p4)
    ex4 = (O.forward(p4, ksub=ks, kernel=(h4, nf4)), O.adjoint(p4, vsub=vs, kernel=(h4, nf4)))
    pairs4 = float(p4.coef.shape[0]) * p4.N * p4.K
    for step in (1, 2, 4):
        wall, f_ms, a_ms, ev, s, z = timed(p4, k4, "closed", step, 1)
        row = {"workload": p4.name, "U": 4, "area_step": step, "ms_per_step": round(wall, 3),
               "ms_forward": round(f_ms, 3), "ms_adjoint": round(a_ms, 3), "pairs_per_s": pairs4 / (wall * 1e-3),
               "area_evaluations": ev,
               "rel_err_vs_exact_oracle": {"forward": rl2(s[:, ks], ex4[0]), "adjoint": rl2(z[:, vs], ex4[1])}}
        if step > 1:
            cg = (O.forward(p4, ksub=ks, kernel=(h4, nf4), step=step),
                  O.adjoint(p4, vsub=vs, kernel=(h4, nf4), step=step))
            row["rel_err_vs_oracle_same_step"] = {"forward": rl2(s[:, ks], cg[0]), "adjoint": rl2(z[:, vs], cg[1])}
        rows[f"coarse_U4_step{step}_fp32"] = row
        log(f"[bench] next coarse grid: {row}")
    return rows


def run_lib(torch, dev, log):
    """The LIB scale (Sec. 2.6), synthesised: 200^3 voxels, 11 520 cylinders,
    L = 2688.  (1) The forward restricted to the nonzero voxels at U = 61 with an
    area per fine bin, in FP64: the paper's exact reference application.  (2)
    The dense A + A^T at U = 11, area per native sample and per fine bin, on a
    sub-scan of one angle x 5 translations (320 cylinders), scaled by K to the
    whole scan: the operator of the paper's reconstruction.  (The forward skips
    the all-zero cubes of the sparse phantom by itself; the adjoint covers every
    voxel.)  Errors against the
    oracle on a few transducers / voxels."""
    import numpy as np
    import oracle as O
    import pat_inputs as P
    from paper_2609_29253_amd.operator import PatOperator

    def rl2(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def events(fn, reps=1):
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(reps):
            out = fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    rows = {}
    p = P.config_lib(U=61)
    nz = int((p.coef != 0).sum())
    log(f"[bench] lib: {p.name} N={p.N} K={p.K} L={p.L} U={p.U}, {nz} nonzero voxels")
    op = PatOperator.from_problem(p, mode="closed", precision="fp64")
    coef = torch.tensor(p.coef, dtype=torch.float64, device=dev)
    ms, s = events(lambda: op.forward(coef, sparse=True))
    ks = np.array([1234, 7777], dtype=np.int32)
    got = s[:, torch.tensor(ks, device=dev).long()].cpu().numpy()
    ws = op.query(5)
    op.close()
    del s, coef
    t = time.perf_counter()
    ref = O.forward(p, ksub=ks)
    log(f"[bench] lib: oracle on transducers {ks.tolist()}: {time.perf_counter() - t:.1f}s")
    pairs = float(nz) * p.K
    rows["lib_sparse_forward_U61_step1_fp64"] = {
        "workload": p.name, "U": p.U, "area_step": 1, "nonzero_voxels": nz, "ms_forward": round(ms, 3),
        "pairs": pairs, "pairs_per_s": pairs / (ms * 1e-3), "workspace_bytes": ws,
        "paper_seconds": 7200.0, "paper_pairs_per_s": 3.8e4,
        "rel_err_vs_oracle": {"forward_transducers": ks.tolist(), "forward": rl2(got, ref)}}
    log(f"[bench] lib sparse forward: {rows['lib_sparse_forward_U61_step1_fp64']}")

    sub = P.config_lib(angles=[0], translations=[0, 3, 7, 11, 14], U=11)
    scale = 11520.0 / sub.K
    ks = np.array([5, 200], dtype=np.int32)
    vs = np.linspace(0, sub.N - 1, 8).astype(np.int64)
    vs[3] = int(np.flatnonzero(sub.coef[0])[0])
    for step, prec in ((11, "fp32"), (11, "fp64"), (1, "fp64")):
        dt = torch.float32 if prec == "fp32" else torch.float64
        op = PatOperator.from_problem(sub, mode="closed", precision=prec, area_step=step)
        coef = torch.tensor(sub.coef, dtype=dt, device=dev)
        y = torch.tensor(sub.y, dtype=dt, device=dev)
        f_ms, s = events(lambda: op.forward(coef))
        a_ms, z = events(lambda: op.adjoint(y))
        evals = op.query(7)
        s = s[:, torch.tensor(ks, device=dev).long()].double().cpu().numpy()
        z = z[:, torch.tensor(vs, device=dev)].double().cpu().numpy()
        op.close()
        del coef, y
        t = time.perf_counter()
        ref = (O.forward(sub, ksub=ks, step=step), O.adjoint(sub, vsub=vs, step=step))
        log(f"[bench] lib: oracle sample {time.perf_counter() - t:.1f}s")
        row = {"workload": sub.name, "U": sub.U, "area_step": step, "transducers": sub.K,
               "ms_forward": round(f_ms, 3), "ms_adjoint": round(a_ms, 3),
               "pairs_per_s": float(sub.N) * sub.K / ((f_ms + a_ms) * 1e-3), "area_evaluations": evals,
               "full_scan_seconds_per_A_AT": round((f_ms + a_ms) * 1e-3 * scale, 2),
               "paper_seconds_per_iteration": 15.8 * 3600 / 30,
               "rel_err_vs_oracle_same_step": {"forward": rl2(s, ref[0]), "adjoint": rl2(z, ref[1])}}
        rows[f"lib_dense_U11_step{step}_{prec}"] = row
        log(f"[bench] lib dense: {row}")
    return rows


def run_pgd(torch, dev, log, ckdir):
    """Config 4's reconstruction at its stated size: 192^3 voxels (0.1 mm), 384
    cylinders (24 elements x 16 rotations), fs 50 MHz, L = 2048, FP32 I/O; y =
    A c_true + 1 % Gaussian noise (relative to max |A c_true|, seed 6) for a
    24-polyline phantom (seed 5); step 0.9 / lambda with lambda the largest
    eigenvalue of A^T A from 20 power iterations (seed 7); c = 0 and 50
    projected-gradient iterations c <- max(0, c - step A^T (A c - y)), a
    checkpoint file every 10 iterations; then a resume from the file of
    iteration 40 through iteration 50, compared with the uninterrupted run."""
    import numpy as np
    import pat_inputs as P
    from paper_2609_29253_amd.operator import (PatOperator, load_checkpoint, power_iteration,
                                               projected_gradient)
    p = P.pgd_cyl384_192c()
    iters = int(p.meta["iterations"])
    log(f"[bench] pgd: {p.name} N={p.N} K={p.K} L={p.L}, {iters} iterations, checkpoints in {ckdir}")
    op = PatOperator.from_problem(p, mode="closed", precision="fp32")
    truth = torch.tensor(p.coef, dtype=torch.float32, device=dev)
    clean = op.forward(truth)
    g = torch.Generator().manual_seed(p.meta["noise_seed"])
    noise = torch.randn(clean.shape, generator=g, dtype=torch.float64).to(dev, torch.float32)
    y = clean + p.meta["noise_level"] * clean.abs().max() * noise
    tn = float(torch.linalg.vector_norm(truth))
    t = time.perf_counter()
    lam = power_iteration(op, iters=20, seed=p.meta["power_seed"])
    t_pow = time.perf_counter() - t
    step = 0.9 / lam
    log(f"[bench] pgd: lambda_max(A^T A) = {lam:.6e} from 20 power iterations in {t_pow:.1f}s, step {step:.6e}")
    marks = {"t": time.perf_counter()}
    times, errs = [], {}

    def cb(it, c, losses):
        now = time.perf_counter()
        times.append(now - marks["t"])
        marks["t"] = now
        if it % 10 == 0 or it == 1:
            errs[it] = float(torch.linalg.vector_norm(c - truth)) / tn
        log(f"[bench] pgd: iteration {it}: loss {losses[-1]:.6e}, {times[-1] * 1e3:.0f} ms"
            + (f", |c - c_true|/|c_true| {errs[it]:.4f}" if it in errs else ""))

    ck = os.path.join(ckdir, "pgd_{it}.pt")
    c, losses = projected_gradient(op, y, iters, step, callback=cb, checkpoint=ck, every=10)
    monotone = all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:]))
    err = float(torch.linalg.vector_norm(c - truth)) / tn
    st = load_checkpoint(ck.replace("{it}", str(iters - 10)))
    t = time.perf_counter()
    c_res, l_res = projected_gradient(op, y, iters, step, state=st)
    t_res = time.perf_counter() - t
    resume_rel = float(torch.linalg.vector_norm(c_res - c) / torch.linalg.vector_norm(c))
    loss_rel = max(abs(a - b) / abs(b) for a, b in zip(l_res[iters - 10:], losses[iters - 10:]))
    op.close()
    it_ms = 1e3 * float(np.median(times))
    row = {"workload": p.name, "voxels": p.N, "transducers": p.K, "samples": p.L, "iterations": iters,
           "io_precision": "fp32", "lambda_max": lam, "step": step, "power_iteration_s": round(t_pow, 2),
           "ms_per_iteration_median": round(it_ms, 1), "ms_per_iteration_mean": round(1e3 * float(np.mean(times)), 1),
           "pairs_per_s_A_plus_AT": float(p.N) * p.K / (it_ms * 1e-3),
           "loss_first": losses[0], "loss_last": losses[-1], "loss_monotone": monotone,
           "rel_err_to_truth_by_iteration": errs, "rel_err_to_truth": err,
           "resume_from_iteration": iters - 10, "resume_s": round(t_res, 2),
           "resume_rel_diff_final_iterate": resume_rel, "resume_max_rel_diff_losses": loss_rel}
    log(f"[bench] pgd: {row}")
    return row


def run_cpu_table(torch, dev, log):
    """Per configuration: the closed form's A + A^T rate on the GPU (FP32 I/O) and
    the oracle's on the host, on all its threads and on one, each over a bounded
    sample (A on a few transducers over every voxel, A^T on a few voxels over
    every transducer), with the GPU / oracle ratio."""
    import numpy as np
    import oracle as O
    from paper_2609_29253_amd.operator import PatOperator
    rows = {}
    threads = O.num_threads()
    for name in ("planar64_32c", "cyl256_128c", "planar512_256c", "batch8_planar256_128c"):
        prob = build_workload(name)
        B = prob.coef.shape[0]
        op = PatOperator.from_problem(prob, mode="closed", precision="fp32", max_batch=B)
        coef = torch.tensor(prob.coef, dtype=torch.float32, device=dev)
        y = torch.tensor(prob.y, dtype=torch.float32, device=dev)
        wall, f_ms, a_ms = time_op(op, coef, y, 2, 1, torch)
        op.close()
        gpu = float(B) * prob.N * prob.K / ((f_ms + a_ms) * 1e-3)
        h, nf = O.kernel_of(prob)

        def rates(nk, nv):
            ks = np.linspace(0, prob.K - 1, nk).astype(np.int32)
            vs = np.linspace(0, prob.N - 1, nv).astype(np.int64)
            t = time.perf_counter()
            O.forward(prob, ksub=ks, kernel=(h, nf))
            tf = time.perf_counter() - t
            t = time.perf_counter()
            O.adjoint(prob, vsub=vs, kernel=(h, nf))
            ta = time.perf_counter() - t
            fw, ad = float(B) * prob.N * nk / tf, float(B) * nv * prob.K / ta
            return {"forward_pairs_per_s": fw, "adjoint_pairs_per_s": ad,
                    "a_plus_at_pairs_per_s": 1.0 / (1.0 / fw + 1.0 / ad),
                    "sample": f"A on {nk} transducers over all voxels ({tf:.1f}s), A^T on {nv} voxels ({ta:.1f}s)"}

        small = prob.N * prob.K < 5e7          # planar64_32c: every transducer, more voxels
        r_all = rates(prob.K if small else threads, 4096 if small else 1024)
        O.set_threads(1)
        r_one = rates(prob.K if small else 1, 1024 if small else 256)
        O.set_threads(threads)
        rows[name] = {"workload": prob.name, "gpu_pairs_per_s": gpu, "oracle_threads": threads,
                      "oracle": r_all, "oracle_1_thread": r_one,
                      "gpu_over_oracle": gpu / r_all["a_plus_at_pairs_per_s"]}
        log(f"[bench] cpu table: {rows[name]}")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cyl256_128c")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib", action="store_true",
                    help="copy a 256 MiB device buffer first (reference kernel for HBM counters)")
    ap.add_argument("--profile-only", action="store_true",
                    help="one forward and one adjoint of the closed FP32 variant, nothing else")
    ap.add_argument("--profile-mode", default="closed", choices=["closed", "quadrature", "trapezoid", "lut"],
                    help="area method of --profile-only")
    ap.add_argument("--probe", action="store_true",
                    help="with --profile-only: also run the FMA probe (its kernels' counters give the clock "
                         "under a pure FMA load for comparison)")
    ap.add_argument("--next", action="store_true",
                    help="also time the approximate variants (trapezoidal and lookup-table cylinder I_l and "
                         "refined quadratures on the workload; the coarse area grid on the 128^3 cylinder "
                         "workload at U = 4) with their errors")
    ap.add_argument("--lib", action="store_true",
                    help="only the LIB-scale rows (sparse forward at U = 61, dense A + A^T at U = 11 on a "
                         "sub-scan), printed as one JSON object instead of the benchmark line")
    ap.add_argument("--pgd", action="store_true",
                    help="only config 4's projected-gradient reconstruction at its stated size (192^3 voxels, "
                         "384 cylinders, 50 iterations, checkpoints every 10, a resume from iteration 40), "
                         "printed as one JSON object instead of the benchmark line")
    ap.add_argument("--tiles", action="store_true",
                    help="only the A/B of the forward's decompositions on the workload (voxel cubes against "
                         "(transducer, time tile) work-groups at several tile widths), printed as one JSON "
                         "object instead of the benchmark line")
    ap.add_argument("--pgd-dir", default=None, help="folder for the --pgd checkpoints (default: a temporary one)")
    ap.add_argument("--cpu-table", action="store_true",
                    help="only the per-configuration GPU and oracle rates (planar64_32c, cyl256_128c, planar512_256c, batch8_planar256_128c), printed as one "
                         "JSON object instead of the benchmark line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the operator is built and timed on a single MI355X; "
              "multi-GPU sharding over transducers is a design note only", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2609_29253_amd.operator import PatOperator, build_kernel

    if args.lib:
        dev = torch.device("cuda", 0)
        print(json.dumps({"lib_rows": run_lib(torch, dev, log)}), flush=True)
        return
    if args.pgd:
        import tempfile
        dev = torch.device("cuda", 0)
        ckdir = args.pgd_dir or tempfile.mkdtemp(prefix="pgd_")
        os.makedirs(ckdir, exist_ok=True)
        print(json.dumps({"pgd": run_pgd(torch, dev, log, ckdir)}), flush=True)
        return
    if args.tiles:
        dev = torch.device("cuda", 0)
        print(json.dumps({"tiles": run_tiles(build_workload(args.workload), torch, dev, log)}), flush=True)
        return
    if args.cpu_table:
        dev = torch.device("cuda", 0)
        print(json.dumps({"cpu_table": run_cpu_table(torch, dev, log)}), flush=True)
        return

    t_build = time.perf_counter()
    prob = build_workload(args.workload)
    log(f"[bench] workload {prob.name}: N={prob.N} K={prob.K} L={prob.L} B={prob.coef.shape[0]} "
        f"({time.perf_counter() - t_build:.1f}s to generate)")
    dev = torch.device("cuda", 0)
    if args.calib:
        xa = torch.empty(1 << 26, dtype=torch.float32, device=dev)
        xb = torch.empty_like(xa)
        xb.copy_(xa)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written")
        del xa, xb
    kern = build_kernel(prob.phi_type, prob.kappa, prob.eir, prob.sound_speed, prob.fs, prob.U)
    B = prob.coef.shape[0]
    pairs = float(B) * prob.N * prob.K
    shapes = set(int(s) for s in prob.tr.packed[:, 0])
    shape = 1 if 1 in shapes else 0

    results = {}

    def run_variant(mode, prec, steps, warmup):
        dt = torch.float32 if prec == "fp32" else torch.float64
        op = PatOperator.from_problem(prob, mode=mode, precision=prec, max_batch=B, kernel=kern)
        coef = torch.tensor(prob.coef, dtype=dt, device=dev)
        y = torch.tensor(prob.y, dtype=dt, device=dev)
        wall, f_ms, a_ms = time_op(op, coef, y, steps, warmup, torch)
        evals = op.query(7)
        s = op.forward(coef)
        z = op.adjoint(y)
        torch.cuda.synchronize()
        out = dict(ms_per_step=wall, ms_forward=f_ms, ms_adjoint=a_ms, evals_per_volume=evals,
                   pairs_per_s=pairs / (wall * 1e-3), s=s.double().cpu().numpy(), z=z.double().cpu().numpy())
        op.close()
        log(f"[bench] {mode}/{prec}: {wall:.2f} ms/step (A {f_ms:.2f} ms, A^T {a_ms:.2f} ms), "
            f"{out['pairs_per_s']:.3e} pairs/s, {evals:.3e} area evaluations per volume")
        return out

    if args.profile_only:
        op = PatOperator.from_problem(prob, mode=args.profile_mode, precision="fp32", max_batch=B, kernel=kern)
        coef = torch.tensor(prob.coef, dtype=torch.float32, device=dev)
        y = torch.tensor(prob.y, dtype=torch.float32, device=dev)
        op.forward(coef)
        op.adjoint(y)
        torch.cuda.synchronize()
        log(f"[bench] profile run done: one A and one A^T of {prob.name} ({args.profile_mode}); "
            f"{op.query(7) * B:.6e} area evaluations per launch")
        op.close()
        if args.probe:
            from paper_2609_29253_amd import _lib
            log(f"[bench] FMA probe: {_lib.probe_peak(0)}")
        return
    main_res = run_variant("closed", "fp32", args.steps, args.warmup)
    results["closed_fp32"] = main_res
    if not args.no_variants:
        for mode, prec in (("closed", "fp64"), ("quadrature", "fp32"), ("quadrature", "fp64")):
            results[f"{mode}_{prec}"] = run_variant(mode, prec, max(1, min(2, args.steps)), 1)

    # ---- roofline of the dominant kernel (the area kernel of A or A^T)
    # the area kernel of A (that of A^T does the same area work and takes the same time)
    dom_ms = main_res["ms_forward"]
    dom_name = "k_fwd_wave"
    dom_full = f"k_fwd_wave<{shape}, {'double' if shape == 1 else 'float'}, {min(B, 8) if B > 1 else 1}, float, 0>"
    area_dtype = "f64" if shape == 1 else "f32"
    evals = main_res["evals_per_volume"] * B
    fl = counter_flops(dom_full, prob.name)
    roofline = {"bound": "alu", "achieved": None, "peak": None, "unit": "TFLOP/s", "frac": None,
                "traffic": measured_traffic(dom_full, prob.name), "kernel": dom_full, "launch_ms": round(dom_ms, 3),
                "area_evaluations_per_launch": evals}
    if fl is not None:
        f64_pe, f32_pe, current, lam = fl
        f64, f32 = f64_pe * evals, f32_pe * evals
        t = dom_ms * 1e-3
        achieved = (f64 + f32) / t / 1e12
        # the peak of this FP64/FP32 mix: the time the published peaks need for it
        peak = (f64 + f32) / (f64 / PEAKS["f64"] + f32 / PEAKS["f32"]) / 1e12
        roofline.update(achieved=round(achieved, 3), peak=round(peak, 2), frac=round(achieved / peak, 4),
                        flops_per_eval={"f64": round(f64_pe, 1), "f32": round(f32_pe, 1)},
                        flops_per_launch=f64 + f32, lane_activity=round(lam, 3),
                        frac_f64=round(f64 / t / PEAKS["f64"], 4), frac_f32=round(f32 / t / PEAKS["f32"], 4),
                        counters_current=current)
    # the published peak placed on this device: an FMA-only kernel built like the library's
    try:
        from paper_2609_29253_amd import _lib
        pk = _lib.probe_peak(0)
        if roofline["achieved"] is not None:
            # the blended mix against the measured FMA ceilings of each precision
            f64_t = roofline["frac_f64"] * PEAKS["f64"] / (pk["fp64_flops"])
            f32_t = roofline["frac_f32"] * PEAKS["f32"] / (pk["fp32_flops"])
            roofline["frac_of_measured_fma_peak"] = round(f64_t + f32_t, 4)
        roofline["device"] = {"compute_units": pk["compute_units"], "clock_ghz": round(pk["clock_ghz"], 3),
                              "fp64_fma_tflops": round(pk["fp64_flops"] / 1e12, 2),
                              "fp32_fma_tflops_unpacked": round(pk["fp32_flops"] / 1e12, 2)}
        log(f"[bench] FMA probe: {roofline['device']}")
    except Exception as exc:   # a measurement aid only; the line stands without it
        log(f"[bench] FMA probe unavailable: {exc}")

    # ---- oracle on the host cores (bounded sample) and accuracy of the sample
    cpu = None
    rel = {}
    if not args.no_cpu:
        import oracle as O
        threads = O.num_threads()
        h, nf = O.kernel_of(prob)
        ks = np.arange(0, prob.K, max(1, prob.K // max(1, threads)))[:max(1, threads)].astype(np.int32)
        t = time.perf_counter()
        s_ref = O.forward(prob, ksub=ks, kernel=(h, nf))
        t_f = time.perf_counter() - t
        f_pairs = float(B) * prob.N * len(ks)
        nv = 2048
        vs = np.linspace(0, prob.N - 1, nv).astype(np.int64)
        t = time.perf_counter()
        z_ref = O.adjoint(prob, vsub=vs, kernel=(h, nf))
        t_a = time.perf_counter() - t
        a_pairs = float(B) * nv * prob.K
        rate = 1.0 / (t_f / f_pairs + t_a / a_pairs)
        # the same oracle on one host thread, on a smaller sample
        O.set_threads(1)
        t = time.perf_counter()
        O.forward(prob, ksub=ks[:1], kernel=(h, nf))
        t_f1 = time.perf_counter() - t
        vs1 = vs[::32]
        t = time.perf_counter()
        O.adjoint(prob, vsub=vs1, kernel=(h, nf))
        t_a1 = time.perf_counter() - t
        O.set_threads(threads)
        rate1 = 1.0 / (t_f1 / (float(B) * prob.N) + t_a1 / (float(B) * len(vs1) * prob.K))
        model = ""
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": rate, "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": f"A on transducers {ks.tolist()} over all {prob.N} voxels ({t_f:.1f}s) and A^T on "
                         f"{nv} evenly spaced voxels over all {prob.K} transducers ({t_a:.1f}s), FP64 surface "
                         f"method; rate = 1/(t_A/pair + t_AT/pair)",
               "value_1_thread": rate1,
               "sample_1_thread": f"A on transducer {int(ks[0])} ({t_f1:.1f}s) and A^T on {len(vs1)} voxels "
                                  f"({t_a1:.1f}s)",
               "cpu_model": model, "host_cpus": os.cpu_count()}
        from numpy.linalg import norm

        def rl2(a, b):
            return float(norm(a - b) / norm(b))

        # quadrature rows are also compared with the oracle's own quadrature
        # (same points: rounding only) on a smaller sample
        qk, qv = ks[:4], vs[::4]
        q_ref = None
        if any(k.startswith("quadrature") for k in results):
            t = time.perf_counter()
            q_ref = (O.forward(prob, ksub=qk, mode=O.MODE_POINT, kernel=(h, nf)),
                     O.adjoint(prob, vsub=qv, mode=O.MODE_POINT, kernel=(h, nf)))
            log(f"[bench] oracle quadrature sample: {time.perf_counter() - t:.1f}s")
        for key, r in results.items():
            # against the FP64 closed-form oracle: rounding for the closed form,
            # method error (plus rounding) for the quadrature
            rel[key] = {"forward": rl2(r["s"][:, ks, :], s_ref), "adjoint": rl2(r["z"][:, vs], z_ref)}
            if key.startswith("quadrature") and q_ref is not None:
                rel[key]["forward_vs_oracle_quadrature"] = rl2(r["s"][:, qk, :], q_ref[0])
                rel[key]["adjoint_vs_oracle_quadrature"] = rl2(r["z"][:, qv], q_ref[1])
        log(f"[bench] oracle: {rate:.3e} pairs/s on {threads} threads; rel errors {rel}")

    next_rows = run_next(args, prob, kern, B, pairs, torch, dev, log) if args.next else None

    value = main_res["pairs_per_s"]
    variants = {k: {"ms_per_step": round(v["ms_per_step"], 3), "pairs_per_s": v["pairs_per_s"],
                    "speedup_of_closed_fp32": round(v["ms_per_step"] / main_res["ms_per_step"], 3)}
                for k, v in results.items()}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-io/" + area_dtype + "-area",
        "data": "synthetic",
        "config": {"workload": prob.name, "voxels": prob.N, "transducers": prob.K, "samples": prob.L,
                   "volumes": B, "U": prob.U, "area": "closed-form", "io_precision": "fp32",
                   "shape": "cylinder" if shape == 1 else "planar"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
        "rel_err_vs_oracle": rel,
    }
    if next_rows is not None:
        line["next_rows"] = next_rows
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
