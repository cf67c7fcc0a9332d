"""Benchmark: FP64 Newton-Schulz sign iteration on a synthetic neighbour-list
Hamiltonian (2048 sites, one 23 x 23 block per site, cutoff 6 A at 0.1
sites/A^3, eps_filter 1e-6, until ||X^2 - I||_F / n < 1e-6), run through the
C ABI on one MI355X.

One step = one whole pass of the path on the device-resident H: X_0 = H/s,
every filtered block-sparse multiply of the iteration, convergence checks,
P = (I - X)/2 and trace(P).  Prints ONE JSON line (rank 0):

    value        algorithmic GFLOP/s of the block products over the whole step
                 (sum of 2 m n k over executed block products / step time)
    ms_per_step  time to the converged sign (+ P and its trace)
    roofline     the block-product kernel: its flops / its HIP-event time vs
                 the FP64 matrix-core peak of MI355X
    cpu_baseline the CPU oracle on a bounded sample of the same workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--seed S]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 matrix (= FP64 vector) peak
PEAK_HBM_GBS = 8000.0
# dense matrix-core peaks of MI355X by the operand type of the block products
PEAK_TFLOPS = {"fp64": PEAK_FP64_TFLOPS, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "split-bf16", "bf16x3": "split-bf16x3"}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(h, rows: int, step_flops: float = 0.0, rows_1t: int = 96):
    """Oracle multiply of the first `rows` block rows of H by H (the first
    product of the sign iteration), timed on the host cores; the same with
    one thread on the first `rows_1t` rows; and the oracle's time to the
    converged sign extrapolated from the measured rate and the step's flops."""
    import numpy as np

    import oracle
    from synth import BSR

    def sample(nrows):
        nnz = int(h.row_ptr[nrows])
        off = h.block_offsets()
        sub = BSR(h.row_blk_size[:nrows], h.col_blk_size, h.row_ptr[:nrows + 1].copy(),
                  h.col_idx[:nnz].copy(), h.values[:off[nnz]].copy())
        lens = np.diff(h.row_ptr)
        b = int(h.row_blk_size[0])
        flops = 2.0 * b ** 3 * int(lens[h.col_idx[:nnz]].sum())
        t0 = time.perf_counter()
        oracle.multiply(1.0, sub, h, eps=1e-6)
        return flops, time.perf_counter() - t0

    threads = oracle.num_threads()
    flops, dt = sample(rows)
    rate = flops / dt
    oracle.set_threads(1)
    try:
        f1, d1 = sample(min(rows_1t, rows))
    finally:
        oracle.set_threads(threads)
    out = dict(value=rate / 1e9, unit="GFLOP/s", cores=threads, kind="oracle",
               sample=f"first {rows} of {h.nbrows} block rows of H*H (the first product of "
                      f"the iteration), eps 1e-6, {flops / 1e9:.1f} GFLOP in {dt:.1f} s; "
                      f"1 thread: first {min(rows_1t, rows)} rows, {f1 / 1e9:.1f} GFLOP in "
                      f"{d1:.1f} s",
               value_1thread=f1 / d1 / 1e9)
    if step_flops > 0.0:
        out["time_to_sign_s_extrapolated"] = step_flops / rate
        out["time_to_sign_note"] = ("the step's algorithmic flops at the sampled oracle rate "
                                    "(extrapolated, not run)")
    return out


KERNEL_SOURCES = ["smm.h", "smm_quad.hip", "quad.hip", "multiply.hip", "graph_iter.hip"]


def sources_sha256() -> str:
    """Hash of the sources that decide the default FP64 block-product
    kernel's memory traffic (the kernel and the order of its work)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2003_03868_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, graph: int):
    """HBM bytes per launch of the block-product kernel from the committed
    rocprofv3 counter summary, or None when the kernel sources have changed
    since the counters were taken, they were taken with another graph mode
    (which changes the launches), or none were taken for this workload."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        d = json.load(open(path))
        sha = sources_sha256()
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != sha or d.get("graph") != graph:
        return None
    return d["hbm_bytes_per_launch"]


def bench_nonorth(args, h, dh, bsm, synth, torch):
    """Timed steps of P = Z (I - sign(Z K Z - mu I)) Z / 2 with Z = S^{-1/2}
    (square root, transforms, sign iteration and back-transform), K = the
    workload's H and a synthetic overlap of its pattern; one JSON line."""
    s = synth.overlap_like(h, args.overlap, seed=args.seed + 1)
    ds = bsm.Matrix.from_bsr(s, device=True)
    torch.cuda.synchronize()
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.order = args.eps, args.tol, args.order
    stream = torch.cuda.current_stream()

    def step():
        st, ph, tps, s1, s2 = bsm.bsm_density_nonorth(dh.handle, ds.handle, 0.0, o, stream=stream)
        if st != bsm.OK:
            raise RuntimeError(f"non-orthogonal density failed: {bsm.STATUS_NAMES[st]} "
                               f"{bsm.bsm_last_error()}")
        bsm.bsm_destroy(ph)
        return s1, s2, tps

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times, recs = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        recs.append(step())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        s1, s2, tps = recs[-1]
        log(f"step {k}: {times[-1] * 1e3:.0f} ms, sqrt {s1.iterations} + sign {s2.iterations} "
            f"iterations, trace(PS)={tps:.6f}, smm {s1.smm_ms + s2.smm_ms:.0f} ms")
    total = sum(times)
    flops = sum(a.flops + b.flops for a, b, _ in recs)
    smm_ms = sum(a.smm_ms + b.smm_ms for a, b, _ in recs)
    s1, s2, tps = recs[-1]
    achieved = flops / (smm_ms * 1e-3) / 1e12 if smm_ms > 0 else 0.0
    print(json.dumps({
        "metric": "block-sparse multiply GFLOP/s (FP64 vs mixed); sign-iteration time to 1e-6",
        "value": flops / total / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 non-orthogonal density matrix (S^-1/2 by coupled "
                               f"Newton-Schulz, sign of S^-1/2 K S^-1/2), {h.nbrows}-site "
                               f"neighbour-list K, overlap S = I + {args.overlap:g} N/M, "
                               f"eps_filter {args.eps:g}, tol {args.tol:g}",
                   "n_sites": h.nbrows, "overlap_tau": args.overlap, "order": args.order,
                   "seed": args.seed},
        "sqrt_iterations": int(s1.iterations), "sign_iterations": int(s2.iterations),
        "multiplies": int(s1.n_multiplies + s2.n_multiplies),
        "trace_ps": float(tps), "n_occ": int(h.meta["n_occ"]),
        "tflop_per_step": flops / args.steps / 1e12,
        "roofline": {"bound": "mfma", "kernel": bsm.bsm_last_smm_kernel(), "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "smm_ms_per_step": smm_ms / args.steps},
        "cpu_baseline": None}))


def bench_mult832(args, bsm, synth, torch):
    """The single FP64 multiply C = A B of 64 x 64 blocks of 13 (832 x 832),
    each block present with probability 0.2, eps 0: repeated calls on the
    resident operands, median per call (the launch- and latency-bound end of
    the range); the oracle times the same multiply on the host."""
    import numpy as np

    import oracle
    a, b = synth.random_bsr_pair(64, 13, 0.2, seed=args.seed)
    da, db = bsm.Matrix.from_bsr(a, device=True), bsm.Matrix.from_bsr(b, device=True)
    dc = bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    stream = torch.cuda.current_stream()
    reps = max(args.steps, 1) * 100
    for _ in range(max(args.warmup, 1) * 10):
        bsm.bsm_multiply(1.0, da.handle, db.handle, 0.0, dc.handle, 0.0, bsm.NORM_FROB,
                         stream=stream)
    torch.cuda.synchronize()
    times, st = [], None
    for _ in range(reps):
        t = time.perf_counter()
        st = bsm.bsm_multiply(1.0, da.handle, db.handle, 0.0, dc.handle, 0.0, bsm.NORM_FROB,
                              stream=stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    med = float(np.median(times))
    kernel_ran = bsm.bsm_last_smm_kernel()

    # Numeric-only repeats of the same multiply from a plan (kernels only: no
    # wait, no allocation), back to back, and the same call captured in a
    # hipGraph and replayed: device time per call between events.
    dp = bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    plan, _ = bsm.bsm_multiply_plan(1.0, da.handle, db.handle, dp.handle, 0.0, stream=stream)
    for _ in range(10):
        bsm.bsm_plan_execute(plan, da.handle, db.handle, dp.handle, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        bsm.bsm_plan_execute(plan, da.handle, db.handle, dp.handle, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    plan_ms = e0.elapsed_time(e1) / reps
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(stream)
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            bsm.bsm_plan_execute(plan, da.handle, db.handle, dp.handle,
                                 stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / reps
    if bsm.bsm_plan_status(plan, stream=stream) != 0:
        raise RuntimeError("planned 832 multiply: the record flags NaN/Inf or another keep-set")
    same = np.array_equal(dp.export()[2], dc.export()[2])
    del g
    bsm.bsm_plan_destroy(plan)
    if not same:
        raise RuntimeError("planned 832 multiply differs from bsm_multiply")

    t0 = time.perf_counter()
    oracle.multiply(1.0, a, b)
    cpu_dt = time.perf_counter() - t0
    achieved = st.flops / (st.smm_ms * 1e-3) / 1e12 if st.smm_ms > 0 else 0.0
    log(f"832 multiply: median {med * 1e3:.3f} ms over {reps} calls, block products "
        f"{st.smm_ms * 1e3:.1f} us, {st.n_products} products; planned repeats "
        f"{plan_ms * 1e3:.1f} us per call, graph replays {graph_ms * 1e3:.1f} us per call")
    print(json.dumps({
        "metric": "block-sparse multiply GFLOP/s (FP64 vs mixed); sign-iteration time to 1e-6",
        "value": st.flops / med / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": reps,
        "warmup": max(args.warmup, 1) * 10, "ms_per_step": med * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 multiply C = A B, 64 x 64 blocks of 13 (832 x 832), "
                               "20% of blocks present, eps_filter 0; median of repeated calls",
                   "seed": args.seed},
        "products": int(st.n_products), "flops": float(st.flops),
        "plan_execute_ms_per_call": plan_ms, "graph_replay_ms_per_call": graph_ms,
        "roofline": {"bound": "mfma", "kernel": kernel_ran,
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "smm_ms_per_step": float(st.smm_ms)},
        "cpu_baseline": {"value": st.flops / cpu_dt / 1e9, "unit": "GFLOP/s",
                         "cores": oracle.num_threads(), "kind": "oracle",
                         "sample": f"the whole multiply, {cpu_dt * 1e3:.1f} ms"}}))


def bench_tc2(args, h, dh, bsm, torch):
    """Timed steps of TC2 or TRS4 purification at the occupied count of the
    workload; one JSON line."""
    name = args.purify.upper()
    fn = bsm.bsm_trs4 if args.purify == "trs4" else bsm.bsm_tc2
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol = args.eps, args.tol
    stream = torch.cuda.current_stream()
    nocc = h.meta["n_occ"]

    def step():
        st, ph, stats = fn(dh.handle, nocc, o, stream=stream)
        if st != bsm.OK:
            raise RuntimeError(f"{name} failed: {bsm.STATUS_NAMES[st]} {bsm.bsm_last_error()}")
        bsm.bsm_destroy(ph)
        return stats

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times, recs = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        recs.append(step())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        s = recs[-1]
        log(f"step {k}: {times[-1] * 1e3:.0f} ms, {s.iterations} iterations, "
            f"e={s.e_hist[s.iterations]:.2e}, trace(P)={s.trace_p:.6f}, smm {s.smm_ms:.0f} ms")
    total = sum(times)
    flops = sum(s.flops for s in recs)
    smm_ms = sum(s.smm_ms for s in recs)
    s = recs[-1]
    achieved = flops / (smm_ms * 1e-3) / 1e12 if smm_ms > 0 else 0.0
    print(json.dumps({
        "metric": "block-sparse multiply GFLOP/s (FP64 vs mixed); sign-iteration time to 1e-6",
        "value": flops / total / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 {name} purification to N = {nocc}, {h.nbrows}-site "
                               f"neighbour-list Hamiltonian, eps_filter {args.eps:g}, "
                               f"tol {args.tol:g}",
                   "n_sites": h.nbrows, "seed": args.seed},
        "iterations": int(s.iterations), "multiplies": int(s.n_multiplies),
        "branches": list(s.branch[:s.iterations]), "trace_p": float(s.trace_p), "n_occ": nocc,
        "gammas": list(s.gamma_hist[:s.iterations]) if args.purify == "trs4" else None,
        "tflop_per_step": flops / args.steps / 1e12,
        "roofline": {"bound": "mfma", "kernel": bsm.bsm_last_smm_kernel(), "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "smm_ms_per_step": smm_ms / args.steps},
        "cpu_baseline": None}))


def bench_submatrix(args, h, dh, bsm, torch):
    """Timed steps of the submatrix method (one dense problem per block
    column); the sparse Newton-Schulz density on the same H timed beside it;
    both measured against a reference P from the sparse iteration with a
    tight filter (untimed).  One JSON line."""
    import math

    import numpy as np
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol = args.eps, args.sub_tol
    stream = torch.cuda.current_stream()
    n = float(h.shape[0])

    def step(keep=False):
        st, ph, stats = bsm.bsm_submatrix_density(dh.handle, 0.0, o, stream=stream)
        if st != bsm.OK:
            raise RuntimeError(f"submatrix failed: {bsm.STATUS_NAMES[st]} {bsm.bsm_last_error()}")
        if keep:
            return stats, ph
        bsm.bsm_destroy(ph)
        return stats

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times, recs = [], []
    ph = None
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        if k == args.steps - 1:
            stats, ph = step(keep=True)
        else:
            stats = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        recs.append(stats)
        log(f"step {k}: {times[-1] * 1e3:.0f} ms, {stats.n_sub} submatrices (max {stats.max_dim}, "
            f"mean {stats.mean_dim:.0f}), {stats.max_iterations} iterations, "
            f"dense products {stats.gemm_ms:.0f} ms, r_max {stats.r_max:.1e}, nnzb(P) {stats.nnzb}")
    total = sum(times)
    flops = sum(s.flops for s in recs)
    gemm_ms = sum(s.gemm_ms for s in recs)
    achieved = flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else 0.0

    # the sparse Newton-Schulz density on the same H and eps (timed alone)
    os_ = bsm.bsm_sign_opts_default()
    os_.eps_filter, os_.tol = args.eps, args.tol
    ns_times = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, xh, sst = bsm.bsm_sign_iterate(dh.handle, 0.0, os_, stream=stream)
        pn, tpn = bsm.bsm_density_from_sign(xh, stream=stream)
        torch.cuda.synchronize()
        ns_times.append(time.perf_counter() - t)
        bsm.bsm_destroy(xh)
        if len(ns_times) < max(1, args.steps):
            bsm.bsm_destroy(pn)
    log(f"sparse Newton-Schulz on the same H: {sum(ns_times) / len(ns_times) * 1e3:.0f} ms, "
        f"{sst.iterations} iterations")

    # reference: sparse iteration with eps 1e-10 (untimed)
    orf = bsm.bsm_sign_opts_default()
    orf.eps_filter, orf.tol = 1e-10, 1e-9
    st, xr, rst = bsm.bsm_sign_iterate(dh.handle, 0.0, orf, stream=stream)
    pr, tpr = bsm.bsm_density_from_sign(xr, stream=stream)
    bsm.bsm_destroy(xr)

    def err(p):
        d = bsm.bsm_add(1.0, p, -1.0, pr, stream=stream)
        num = bsm.bsm_sqdist_identity(d, 0.0, stream=stream)
        bsm.bsm_destroy(d)
        return math.sqrt(num / bsm.bsm_sqdist_identity(pr, 0.0, stream=stream))

    tp_sub = bsm.bsm_trace(ph, stream=stream)
    e_sub, e_ns = err(ph), err(pn)
    log(f"vs reference (sparse, eps 1e-10): submatrix {e_sub:.2e} (trace {tp_sub - tpr:+.2e}), "
        f"Newton-Schulz {e_ns:.2e} (trace {tpn - tpr:+.2e})")
    for hnd in (ph, pn, pr):
        bsm.bsm_destroy(hnd)

    cpu = None
    if not args.no_cpu:
        import oracle
        cols = np.random.default_rng(0).choice(h.nbrows, min(args.cpu_cols, h.nbrows), replace=False)
        t0 = time.perf_counter()
        _, rec = oracle.submatrix_density(h, columns=cols)
        dt = time.perf_counter() - t0
        cpu = dict(value=len(cols) / (dt * h.nbrows), unit="P/s (whole matrix)",
                   cores=oracle.num_threads(), kind="oracle",
                   sample=f"{len(cols)} of {h.nbrows} block columns (dense eigendecomposition of "
                          f"each submatrix, mean edge {np.mean(rec['dims']):.0f}) in {dt:.1f} s, "
                          f"scaled to all columns: {dt * h.nbrows / len(cols):.1f} s per P")
        log(f"cpu baseline: {cpu['sample']}")

    s0 = recs[-1]
    print(json.dumps({
        "metric": "block-sparse multiply GFLOP/s (FP64 vs mixed); sign-iteration time to 1e-6",
        "value": flops / total / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 submatrix-method density, {h.nbrows}-site neighbour-list "
                               f"Hamiltonian, {int(h.row_blk_size[0])}x{int(h.row_blk_size[0])} "
                               f"blocks, {args.density:g} sites/A^3, cutoff {args.cutoff:g} A, "
                               f"eps_filter {args.eps:g}, submatrix tol {args.sub_tol:g}",
                   "n_sites": h.nbrows, "n": int(n), "nnzb_H": h.nnzb, "seed": args.seed},
        "time_to_P_ms": total / args.steps * 1e3,
        "n_sub": int(s0.n_sub), "max_dim": int(s0.max_dim), "mean_dim": float(s0.mean_dim),
        "iterations_max": int(s0.max_iterations), "r_max": float(s0.r_max),
        "tflop_per_step": flops / args.steps / 1e12,
        "rel_err_vs_reference": e_sub, "trace_diff_vs_reference": tp_sub - tpr,
        "newton_schulz_same_H": {"ms": sum(ns_times) / len(ns_times) * 1e3,
                                 "iterations": int(sst.iterations), "rel_err_vs_reference": e_ns,
                                 "trace_diff_vs_reference": tpn - tpr},
        "roofline": {"bound": "mfma", "kernel": "k_sub_gemm", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "gemm_ms_per_step": gemm_ms / args.steps},
        "cpu_baseline": cpu}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", choices=["sign23", "mixed", "mult832", "water"], default="sign23",
                    help="sign23: 2048 sites x 23; mixed: 4096 sites, sizes {5,13,23,26}; "
                         "mult832: one 832 x 832 multiply (64 x 64 blocks of 13, 20%% present); "
                         "water: 6192 sites x 6 at 0.0334 sites/A^3 (water-like, minimal basis)")
    ap.add_argument("--sites", type=int, default=0, help="override the site count")
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cpu-rows", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16", "bf16x3"], default="fp64",
                    help="block-product precision: fp32, split-bf16 with two (bf16) or three "
                         "(bf16x3) parts per operand; all switch to FP64 once r_k < 1e-4")
    ap.add_argument("--table", choices=["exhaustive", "mlp", "mlp_raw", "none"], default="exhaustive",
                    help="kernel-parameter table: measured (exhaustive autotuning), predicted "
                         "by the MLP ensemble (exhaustive where its members disagree; mlp_raw: "
                         "the prediction everywhere), or none (built-in choices)")
    ap.add_argument("--order", type=int, choices=[2, 3, 5, 7], default=2,
                    help="sign iteration order: 2 Newton-Schulz, 3, 5 (four multiplies per iteration)")
    ap.add_argument("--overlap", type=float, default=0.0, metavar="TAU",
                    help="time the non-orthogonal density matrix with a synthetic overlap "
                         "S = I + TAU N/M (0: the orthogonal sign iteration)")
    ap.add_argument("--purify", choices=["sign", "tc2", "trs4"], default="sign",
                    help="density matrix by the sign iteration (default) or by TC2 or TRS4 "
                         "purification at the occupied count")
    ap.add_argument("--screen", type=float, default=0.0, metavar="TAU",
                    help="leave out block products with ||A_ik|| ||B_kj|| < TAU in the "
                         "Newton-Schulz multiplies (FP64, order 2)")
    ap.add_argument("--method", choices=["sign", "submatrix"], default="sign",
                    help="submatrix: the submatrix method (dense problem per block column) "
                         "on the water-like workload unless --workload says otherwise")
    ap.add_argument("--sub-tol", type=float, default=1e-8,
                    help="Newton-Schulz tolerance inside each submatrix")
    ap.add_argument("--cpu-cols", type=int, default=1500,
                    help="block columns of the oracle's submatrix sample")
    ap.add_argument("--mixed-kernel", choices=["fused", "class"], default="fused",
                    help="mixed workload: every (m, n) class in one persistent launch per "
                         "multiply with operand sharing (fused, the configuration's form) or "
                         "one launch per class (the library default, measured faster)")
    ap.add_argument("--graph", type=int, choices=[0, 1, 2], default=1,
                    help="1 (default): iterations from captured hipGraphs of the whole "
                         "device-sized multiply once X's block count settles; 2: replay of "
                         "the numeric kernels once X's block pattern stops changing; 0: none")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU "
                                   "sharding is a design (block rows of C per GPU), "
                                   "not part of this build", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        # A plain copy of known size: each dispatch reads and writes exactly
        # MIB MiB, which scales the HBM read/write counters of the profiler.
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.randn(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_mib": args.calibrate_copy, "dispatches": 5}))
        return

    if args.workload == "mixed" and args.mixed_kernel == "fused" and "BSM_SMM_VARIANT" not in os.environ:
        os.environ["BSM_SMM_VARIANT"] = "7"      # read by the library per multiply
    import synth
    from paper_2003_03868_amd import bsm, tune
    bsm.load()
    torch.cuda.set_device(0)
    tune.install_default(args.table)

    if args.workload == "mult832":
        bench_mult832(args, bsm, synth, torch)
        return

    if args.method == "submatrix" and args.workload == "sign23" and "--workload" not in sys.argv:
        args.workload = "water"
    args.density, args.cutoff = 0.1, 6.0
    t0 = time.perf_counter()
    if args.workload == "water":
        args.sites = args.sites or 6192
        args.density = 0.0334
        h = synth.neighbour_hamiltonian(args.sites, 6, density=args.density, cutoff=args.cutoff,
                                        seed=args.seed)
    elif args.workload == "sign23":
        args.sites = args.sites or 2048
        h = synth.neighbour_hamiltonian(args.sites, 23, density=0.1, cutoff=6.0, seed=args.seed)
    else:
        args.sites = args.sites or 4096
        h = synth.neighbour_hamiltonian(args.sites, density=0.1, cutoff=6.0, seed=args.seed,
                                        size_choices=(5, 13, 23, 26))
    log(f"generated H: {h.nbrows} sites, {h.nnzb} blocks, n_occ {h.meta['n_occ']} "
        f"({time.perf_counter() - t0:.1f} s)")
    dh = bsm.Matrix.from_bsr(h, device=True)
    torch.cuda.synchronize()

    if args.method == "submatrix":
        bench_submatrix(args, h, dh, bsm, torch)
        return
    if args.overlap > 0.0:
        bench_nonorth(args, h, dh, bsm, synth, torch)
        return
    if args.purify in ("tc2", "trs4"):
        bench_tc2(args, h, dh, bsm, torch)
        return

    opts = bsm.bsm_sign_opts_default()
    opts.eps_filter = args.eps
    opts.tol = args.tol
    opts.prec = {"fp64": bsm.FP64, "fp32": bsm.FP32, "bf16": bsm.SPLIT_BF16,
                 "bf16x3": bsm.SPLIT_BF16X3}[args.prec]
    opts.use_graph = args.graph
    opts.order = args.order
    opts.eps_screen = args.screen
    stream = torch.cuda.current_stream()

    def step(keep=False):
        st, xh, stats = bsm.bsm_sign_iterate(dh.handle, 0.0, opts, stream=stream)
        if st != bsm.OK:
            raise RuntimeError(f"sign iteration failed: {bsm.STATUS_NAMES[st]} "
                               f"{bsm.bsm_last_error()}")
        ph, tp = bsm.bsm_density_from_sign(xh, stream=stream)
        if keep:
            return stats, tp, xh, ph
        bsm.bsm_destroy(ph)
        bsm.bsm_destroy(xh)
        return stats, tp

    for w in range(args.warmup):
        stats, tp = step()
        log(f"warmup {w}: {stats.iterations} iterations, {stats.flops / 1e12:.2f} TFLOP, "
            f"device {stats.device_ms:.0f} ms")

    torch.cuda.synchronize()
    times, all_stats = [], []
    xd = pd = None
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        if k == args.steps - 1:
            stats, tp, xd, pd = step(keep=True)   # the last iterate feeds the diagnostics
        else:
            stats, tp = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        all_stats.append((stats, tp))
        log(f"step {k}: {times[-1] * 1e3:.0f} ms, {stats.iterations} iterations, "
            f"r={stats.r_hist[stats.iterations]:.2e}, trace(P)={tp:.6f}, "
            f"smm {stats.smm_ms:.0f} ms in {stats.smm_launches} launches, nnzb(X)={stats.nnzb_final}, "
            f"graph replays {stats.graph_replays} (fallbacks {stats.graph_fallbacks})")
    total = sum(times)
    flops = sum(s.flops for s, _ in all_stats)
    smm_ms = sum(s.smm_ms for s, _ in all_stats)
    s0, tp0 = all_stats[-1]

    # the block-product kernel of this configuration, as the library reports
    # launching it (one untimed H H multiply at the run's precision)
    hh = bsm.Matrix.empty_like(h.row_blk_size, h.col_blk_size)
    if args.screen > 0.0:
        bsm.bsm_multiply_screened(1.0, dh.handle, dh.handle, 0.0, hh.handle, args.eps,
                                  bsm.NORM_FROB, args.screen, stream=stream)
    else:
        bsm.bsm_multiply(1.0, dh.handle, dh.handle, 0.0, hh.handle, args.eps, bsm.NORM_FROB,
                         opts.prec, stream=stream)
    kernel_ran = bsm.bsm_last_smm_kernel()
    if kernel_ran.startswith("k_smm_f64_class<"):
        kernel_ran = "k_smm_f64_class<m, n> (one launch per (m, n) class)"
    hh.destroy()
    ms_per_step = total / args.steps * 1e3
    achieved = flops / (smm_ms * 1e-3) / 1e12 if smm_ms > 0 else 0.0

    # density-matrix diagnostic of the last step's iterate (untimed):
    # idempotency ||P^2 - P||_F / n on the device, P^2 filtered like every product
    import math
    p2 = bsm.Matrix.empty_like(h.row_blk_size, h.col_blk_size)
    bsm.bsm_multiply(1.0, pd, pd, 0.0, p2.handle, args.eps, bsm.NORM_FROB, stream=stream)
    dd = bsm.bsm_add(1.0, p2.handle, -1.0, pd, stream=stream)
    idem = math.sqrt(bsm.bsm_sqdist_identity(dd, 0.0, stream=stream)) / float(h.shape[0])
    for hnd in (dd, pd):
        bsm.bsm_destroy(hnd)
    p2.destroy()
    log(f"||P^2 - P||_F / n = {idem:.3e}")

    err64 = None
    if args.prec != "fp64" or args.screen > 0.0:
        # error of the reduced-precision or screened sign against the plain
        # FP64 GPU path on the same input (untimed): ||X_p - X_64||_F / ||X_64||_F
        # and trace(P)
        xp, sp = xd, s0
        o64 = bsm.bsm_sign_opts_default()
        for f, _ in bsm.bsm_sign_opts._fields_:
            setattr(o64, f, getattr(opts, f))
        o64.prec = bsm.FP64
        o64.eps_screen = 0.0
        st_64, x64, s64 = bsm.bsm_sign_iterate(dh.handle, 0.0, o64, stream=stream)
        if st_64 != bsm.OK:
            raise RuntimeError(f"FP64 reference sign iteration failed: {bsm.STATUS_NAMES[st_64]} "
                               f"{bsm.bsm_last_error()}")
        d = bsm.bsm_add(1.0, xp, -1.0, x64, stream=stream)
        num = bsm.bsm_sqdist_identity(d, 0.0, stream=stream)
        den = bsm.bsm_sqdist_identity(x64, 0.0, stream=stream)
        err64 = {"rel_fro_X_vs_fp64": math.sqrt(num / den), "trace_p": float(sp.trace_p),
                 "trace_p_fp64": float(s64.trace_p),
                 "trace_p_diff": float(sp.trace_p - s64.trace_p),
                 "precisions": list(sp.prec_hist[:sp.iterations + 1])}
        for hnd in (d, x64):
            bsm.bsm_destroy(hnd)
        log(f"error vs FP64 path: {err64}")
    bsm.bsm_destroy(xd)

    cpu = None
    if not args.no_cpu and args.workload == "sign23":
        log("timing the CPU oracle on a sample ...")
        cpu = cpu_baseline(h, min(args.cpu_rows, h.nbrows),
                           step_flops=sum(s.flops for s, _ in all_stats) / args.steps)
        # the oracle's own run of this whole sign iteration, when its record
        # (tests/golden, written on the build host) is for this configuration
        rec = os.path.join(ROOT, "tests", "golden", f"fullsize_sign23_s{args.seed}.npz")
        if (os.path.exists(rec) and args.sites == 2048 and args.eps == 1e-6 and args.tol == 1e-6
                and args.order == 2 and args.prec == "fp64" and args.screen == 0.0):
            with np.load(rec, allow_pickle=False) as z:
                cpu["time_to_sign_s_oracle_record"] = float(z["oracle_seconds"])
                cpu["oracle_record_threads"] = int(z["oracle_threads"])
                cpu["oracle_record_note"] = "measured once on the build host when the record was written"
        log(f"cpu baseline: {cpu['value']:.2f} GFLOP/s on {cpu['cores']} threads")

    n = float(h.shape[0])
    out = {
        "metric": "block-sparse multiply GFLOP/s (FP64 vs mixed); sign-iteration time to 1e-6",
        "value": flops / total / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {
            "workload": (f"{args.prec.upper()} {'Newton-Schulz' if args.order == 2 else f'order-{args.order}'} sign iteration, {h.nbrows}-site "
                         "neighbour-list Hamiltonian, "
                         + {"sign23": "23x23 blocks", "water": "6x6 blocks"}.get(
                             args.workload, "block sizes {5,13,23,26}") +
                         f", cutoff {args.cutoff:g} A, {args.density:g} sites/A^3, "
                         f"eps_filter {args.eps:g}, to ||X^2-I||_F/n < {args.tol:g}"),
            "n_sites": h.nbrows,
            "block": {"sign23": 23, "water": 6}.get(args.workload, "5/13/23/26"),
            "n": int(n), "eps_filter": args.eps, "kernel_table": args.table,
            "tol": args.tol, "seed": args.seed, "nnzb_H": h.nnzb,
            "graph_mode": args.graph, "order": args.order,
            "mixed_kernel": (args.mixed_kernel if args.workload == "mixed" else None),
            "eps_screen": args.screen,
        },
        "time_to_sign_ms": ms_per_step,
        "iterations": int(s0.iterations),
        "multiplies": int(s0.n_multiplies),
        "smm_launches_per_step": int(s0.smm_launches),
        "r_final": float(s0.r_hist[s0.iterations]),
        "trace_p": float(tp0),
        "n_occ": int(h.meta["n_occ"]),
        "tflop_per_step": flops / args.steps / 1e12,
        "products_per_step": int(sum(s.n_products for s, _ in all_stats) / args.steps),
        "products_screened_per_step": int(sum(s.n_screened for s, _ in all_stats) / args.steps),
        "nnzb_X_final": int(s0.nnzb_final),
        "idempotency_P": idem,
        "graph_replays": int(s0.graph_replays),
        "graph_fallbacks": int(s0.graph_fallbacks),
        "roofline": {
            "bound": "mfma",
            "kernel": kernel_ran,
            "achieved": achieved,
            "peak": PEAK_TFLOPS[args.prec],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[args.prec],
            "traffic": measured_traffic("sign23", args.graph)
            if (args.prec == "fp64" and args.workload == "sign23" and args.sites == 2048
                and args.eps == 1e-6 and args.table == "exhaustive" and args.screen == 0.0)
            else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, "
                            "profiles/k_smm_f64_quad_sign23.md)",
            "smm_ms_per_step": smm_ms / args.steps,
        },
        "cpu_baseline": cpu,
    }
    if err64 is not None:
        out["error_vs_fp64"] = err64
    print(json.dumps(out), flush=True)
    dh.destroy()


if __name__ == "__main__":
    main()
