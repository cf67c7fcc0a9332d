"""End-to-end parity of the benchmarked sign iterations at full size against
the oracle's stored record.

The records (``tests/golden/fullsize_<workload>_s<seed>.npz``) are written by
``tests/golden/make_fullsize.py``, which runs only the CPU oracle on the same
seeded workloads (2048 sites x 23 with eps_filter 1e-6 and 1e-5, and with
the third- and fifth-order iterations; 4096 sites of sizes {5, 13, 23, 26}).
The GPU runs ``bsm_sign_iterate`` with the benchmark's settings (default
kernels, chunking and options, iterations from the device-sized graphs;
sign23 seed 0 also without graphs) and must give:

* the same number of iterations and, at every iterate, the same number of
  stored blocks of X_k and of Y_k = filter(X_k X_k) (Sign-Method section:
  filtering after every product), and the same block pattern of the
  returned X (SHA-256 of row_ptr and col_idx);
* r_k within a relative 1e-6 of the oracle's at every k;
* X within 1e-10 relative Frobenius error of the oracle's, estimated by
  Gaussian probe vectors v (E||(X' - X) v||^2 = ||X' - X||_F^2), and the
  squared Frobenius norm of every block row within 2e-10 (relative, over
  all rows);
* trace(P) within the bound the Frobenius tolerance implies,
  |tr(X' - X)| <= sqrt(n) ||X' - X||_F, halved for P = (I - X)/2.

The reduced-precision forms (FP32, split-BF16 with three terms) are held to
1e-6 relative Frobenius error of the FP64 oracle on the eps 1e-5 workload,
and trace(P) to the bound 1e-6 implies; the two-term split-BF16 form is
reported against the same record and held to its own measured level.
"""
import math

import numpy as np
import pytest

import synth
from tests.gpu_util import TOL_FP64, TOL_MIXED, need_gpu
from tests.golden.make_fullsize import (WORKLOADS, hamiltonian, load_fixture, pattern_digest,
                                        sketch)

pytestmark = pytest.mark.gpu

# (workload, seed, kernel variant, graph mode): the mixed workload both with
# the paired-group kernel in one launch per multiply (bench.py --workload
# mixed) and with the library default, one launch per (m, n) class
CASES = [("sign23", 0, None, 1), ("sign23", 0, None, 0), ("sign23", 1, None, 1),
         ("sign23", 2, None, 1), ("sign23_e5", 0, None, 1), ("mixed", 0, "7", 1),
         ("mixed", 0, "4", 1), ("mixed", 1, "7", 1), ("sign23_o3", 0, None, 1),
         ("sign23_o5", 0, None, 1)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _fixture(workload, seed):
    fx = load_fixture(workload, seed)
    if fx is None:
        pytest.skip(f"oracle record for {workload} seed {seed} has not been written")
    return fx


def _sign(h, workload, prec=0, graph=1):
    from paper_2003_03868_amd import bsm
    from tests.gpu_util import from_dev, to_dev
    w = WORKLOADS[workload]
    dh = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.prec, o.use_graph = w["eps"], w["tol"], prec, graph
    o.order = w.get("order", 2)
    print(f"sign iteration: {workload}, {h.nbrows} sites, order {o.order}, prec {prec}, "
          f"graph mode {graph}", flush=True)
    st, xh, stats = bsm.bsm_sign_iterate(dh.handle, 0.0, o)
    assert st == bsm.OK, bsm.bsm_last_error()
    x = from_dev(bsm.Matrix(xh, h.row_blk_size, h.col_blk_size))
    dh.destroy()
    return x, stats


def _probe_err(x, fx):
    v = synth.probe_vectors(x.shape[0], fx["xv"].shape[0], int(fx["probe_seed"]))
    xv, row_sq = sketch(x, v)
    ref = fx["xv"]
    errs = [float(np.linalg.norm(xv[q] - ref[q]) / np.linalg.norm(ref[q]))
            for q in range(ref.shape[0])]
    row_err = float(np.linalg.norm(row_sq - fx["row_sqnorm"]) / np.linalg.norm(fx["row_sqnorm"]))
    return errs, row_err


@pytest.mark.parametrize("workload,seed,variant,graph", CASES,
                         ids=[f"{w}-s{s}" + (f"-v{v}" if v else "") + f"-g{g}"
                              for w, s, v, g in CASES])
def test_sign_full_size_matches_oracle(monkeypatch, workload, seed, variant, graph):
    fx = _fixture(workload, seed)
    if variant is not None:
        monkeypatch.setenv("BSM_SMM_VARIANT", variant)
    h = hamiltonian(workload, seed)
    assert h.nbrows == int(fx["sites"])
    x, st = _sign(h, workload, graph=graph)
    k = int(fx["iterations"])
    assert st.iterations == k, (st.iterations, k)
    gx = np.array(st.nnzb_x_hist[:k + 1])
    gy = np.array(st.nnzb_y_hist[:k + 1])
    assert np.array_equal(gx, fx["nnzb_x"]), (gx, fx["nnzb_x"])
    assert np.array_equal(gy, fx["nnzb_y"]), (gy, fx["nnzb_y"])
    r = np.array(st.r_hist[:k + 1])
    assert np.allclose(r, fx["r_hist"], rtol=1e-6, atol=0.0), (r, fx["r_hist"])
    assert x.nnzb == int(fx["nnzb_final"])
    assert pattern_digest(x) == str(fx["pattern_sha256"]), "block pattern of X differs"
    errs, row_err = _probe_err(x, fx)
    assert max(errs) <= TOL_FP64, errs
    assert row_err <= 2 * TOL_FP64, row_err
    n = float(h.shape[0])
    x_fro = math.sqrt(float(fx["row_sqnorm"].sum()))
    trace_bound = 0.5 * math.sqrt(n) * TOL_FP64 * x_fro
    dtr = abs(st.trace_p - float(fx["trace_p"]))
    assert dtr <= trace_bound, (dtr, trace_bound)
    print(f"{workload} seed {seed}: {k} iterations ({st.graph_replays} from graphs), "
          f"nnzb(X) {x.nnzb}, probe errors "
          f"{max(errs):.2e}, row-norm error {row_err:.2e}, |dtrace(P)| {dtr:.2e} "
          f"(bound {trace_bound:.1e}), max r_k rel diff "
          f"{float(np.max(np.abs(r / fx['r_hist'] - 1))):.1e}")


@pytest.mark.parametrize("prec,tol", [(1, TOL_MIXED), (3, TOL_MIXED), (2, 4e-6)],
                         ids=["fp32", "split_bf16x3", "split_bf16x2"])
def test_reduced_precision_full_size_vs_oracle(prec, tol):
    """The reduced-precision workload (2048 sites x 23, eps_filter 1e-5):
    sign(H) from FP32 / split-BF16 block products with FP64 refinement,
    against the FP64 oracle.  The two-term split keeps about 17 bits per
    operand and is held to its measured level, above the 1e-6 target."""
    fx = _fixture("sign23_e5", 0)
    h = hamiltonian("sign23_e5", 0)
    x, st = _sign(h, "sign23_e5", prec)
    errs, row_err = _probe_err(x, fx)
    n = float(h.shape[0])
    x_fro = math.sqrt(float(fx["row_sqnorm"].sum()))
    dtr = abs(st.trace_p - float(fx["trace_p"]))
    precs = list(st.prec_hist[:st.iterations + 1])
    print(f"prec {prec}: {st.iterations} iterations (products {precs}), probe errors "
          f"{[f'{e:.2e}' for e in errs]}, |dtrace(P)| {dtr:.2e}")
    assert max(errs) <= tol, errs
    assert dtr <= 0.5 * math.sqrt(n) * tol * x_fro, dtr
