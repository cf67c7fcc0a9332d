"""Full-size oracle fixtures of the sign iteration (test data writer).

Runs only the CPU oracle (``oracle/``) on the seeded synthetic workloads that
the benchmark times, and stores a compact record of the result that the GPU
parity test (``tests/test_gpu_fullsize_oracle.py``) compares against:

* the iteration count, the residual history r_k = ||X_k^2 - I||_F / n and the
  number of stored blocks of every X_k and Y_k = filter(X_k X_k)
  (Sign-Method section: Eq. signdef, filtering after every product);
* trace(X) and trace(P) of the returned iterate (the density-matrix relation);
* a SHA-256 digest of the returned X's block pattern (row_ptr as int64,
  col_idx as int32, little-endian);
* the squared Frobenius norm of every block row of X;
* X V for seeded Gaussian probe vectors V (``synth.probe_vectors``), which
  sketches X: for Gaussian v, E||(X' - X) v||^2 = ||X' - X||_F^2.

Workloads (``--workload``):

* ``sign23``    -- 2048 sites x 23, density 0.1 / A^3, cutoff 6 A,
                   eps_filter 1e-6, tol 1e-6;
* ``sign23_e5`` -- the same H with eps_filter 1e-5 (the reduced-precision
                   workload's filter);
* ``mixed``     -- 4096 sites, block sizes {5, 13, 23, 26}, eps 1e-6, tol 1e-6;
* ``sign23_o3``, ``sign23_o5`` -- sign23's H and filter with the third- and
                   fifth-order iterations (the paper's higher-order updates).

Usage (CPU only; hours at full size on a few cores)::

    python tests/golden/make_fullsize.py --workload sign23 --seed 0

writes ``tests/golden/fullsize_<workload>_s<seed>.npz``.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

N_PROBES = 2

WORKLOADS = {
    "sign23": dict(sites=2048, block=23, eps=1e-6, tol=1e-6),
    "sign23_e5": dict(sites=2048, block=23, eps=1e-5, tol=1e-6),
    "mixed": dict(sites=4096, block=None, eps=1e-6, tol=1e-6),
    "sign23_o3": dict(sites=2048, block=23, eps=1e-6, tol=1e-6, order=3),
    "sign23_o5": dict(sites=2048, block=23, eps=1e-6, tol=1e-6, order=5),
}


def hamiltonian(workload: str, seed: int, scale: float = 1.0) -> synth.BSR:
    """The workload's H (the benchmark's generator call)."""
    w = WORKLOADS[workload]
    sites = max(8, int(round(w["sites"] * scale)))
    if w["block"] is None:
        return synth.neighbour_hamiltonian(sites, density=0.1, cutoff=6.0, seed=seed,
                                           size_choices=(5, 13, 23, 26))
    return synth.neighbour_hamiltonian(sites, w["block"], density=0.1, cutoff=6.0, seed=seed)


def probe_seed(seed: int) -> int:
    return 1000 + seed


def fixture_path(workload: str, seed: int) -> str:
    return os.path.join(HERE, f"fullsize_{workload}_s{seed}.npz")


def pattern_digest(m: synth.BSR) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(m.row_ptr, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(m.col_idx, dtype="<i4").tobytes())
    return h.hexdigest()


def sketch(m: synth.BSR, v: np.ndarray, chunk: int = 1 << 17):
    """(X V^T as rows, squared Frobenius norm per block row) of a BSR matrix,
    block by block in chunks (no dense copy)."""
    rows = m.block_rows()
    off = m.block_offsets()
    rbs, cbs = m.row_blk_size.astype(np.int64), m.col_blk_size.astype(np.int64)
    r_off = np.concatenate([[0], np.cumsum(rbs)])
    c_off = np.concatenate([[0], np.cumsum(cbs)])
    n_rows = int(r_off[-1])
    p = v.shape[0]
    y = np.zeros((p, n_rows))
    row_sq = np.zeros(m.nbrows)
    shapes = np.stack([rbs[rows], cbs[m.col_idx]], 1) if m.nnzb else np.zeros((0, 2), np.int64)
    for mm, nn in sorted(set(map(tuple, shapes.tolist()))):
        sel_all = np.nonzero((shapes[:, 0] == mm) & (shapes[:, 1] == nn))[0]
        for s in range(0, sel_all.size, chunk):
            sel = sel_all[s:s + chunk]
            vi = off[sel][:, None] + np.arange(mm * nn)[None, :]
            blk = m.values[vi].reshape(-1, mm, nn)
            row_sq += np.bincount(rows[sel], weights=(blk * blk).sum((1, 2)), minlength=m.nbrows)
            ci = c_off[m.col_idx[sel]][:, None] + np.arange(nn)[None, :]      # (b, nn)
            ri = (r_off[rows[sel]][:, None] + np.arange(mm)[None, :]).ravel()
            for q in range(p):
                contrib = np.matmul(blk, v[q][ci][:, :, None])[:, :, 0]       # (b, mm)
                y[q] += np.bincount(ri, weights=contrib.ravel(), minlength=n_rows)
    return y, row_sq


def load_fixture(workload: str, seed: int):
    """The stored record as a dict, or None when it has not been written."""
    path = fixture_path(workload, seed)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="sign23")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="site-count factor (< 1 for a quick trial; not a fixture)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import oracle
    oracle.build(force=False)
    w = WORKLOADS[args.workload]
    h = hamiltonian(args.workload, args.seed, args.scale)
    print(f"{args.workload} seed {args.seed}: {h.nbrows} sites, {h.nnzb} blocks, "
          f"n = {h.shape[0]}, oracle threads {oracle.num_threads()}", flush=True)
    t0 = time.time()
    x, st, status = oracle.sign_ns(h, eps=w["eps"], tol=w["tol"], order=w.get("order", 2))
    dt = time.time() - t0
    if status != oracle.OK:
        raise SystemExit(f"oracle sign iteration ended with status {status}")
    print(f"  {st['iterations']} iterations, {st['n_multiplies']} multiplies, "
          f"{st['flops'] / 1e12:.1f} TFLOP in {dt:.0f} s; trace(P) {st['trace_p']:.9f}", flush=True)
    v = synth.probe_vectors(h.shape[0], N_PROBES, probe_seed(args.seed))
    xv, row_sq = sketch(x, v)
    out = args.out or fixture_path(args.workload, args.seed)
    np.savez_compressed(
        out, workload=np.array(args.workload), seed=np.int64(args.seed),
        sites=np.int64(h.nbrows), eps=np.float64(w["eps"]), tol=np.float64(w["tol"]),
        order=np.int64(w.get("order", 2)),
        iterations=np.int64(st["iterations"]), n_multiplies=np.int64(st["n_multiplies"]),
        r_hist=np.array(st["r_hist"]), nnzb_x=np.array(st["nnzb_x"], np.int64),
        nnzb_y=np.array(st["nnzb_y"], np.int64), trace_x=np.float64(st["trace_x"]),
        trace_p=np.float64(st["trace_p"]), flops=np.float64(st["flops"]),
        nnzb_final=np.int64(x.nnzb), pattern_sha256=np.array(pattern_digest(x)),
        row_sqnorm=row_sq, probe_seed=np.int64(probe_seed(args.seed)), xv=xv,
        oracle_seconds=np.float64(dt), oracle_threads=np.int64(oracle.num_threads()))
    print(f"  wrote {out}", flush=True)


if __name__ == "__main__":
    main()
