"""CPU checks of the full-size oracle records and of the sketch that the GPU
parity test compares them with (tests/golden/make_fullsize.py)."""
import numpy as np
import pytest

import synth
from tests.golden.make_fullsize import (WORKLOADS, fixture_path, hamiltonian, load_fixture,
                                        pattern_digest, sketch)


def test_sketch_matches_dense_product():
    """X V and the block-row norms of a mixed-size matrix, against the dense
    matrix (chunks smaller than the block count)."""
    rng = np.random.default_rng(3)
    sz = rng.choice([5, 13, 23, 26], 17).astype(np.int32)
    m = synth.random_bsr(17, 17, sz, sz, 0.4, rng)
    v = synth.probe_vectors(m.shape[0], 3, 9)
    y, row_sq = sketch(m, v, chunk=7)
    d = m.to_dense()
    assert np.allclose(y, (d @ v.T).T, rtol=1e-13, atol=1e-12)
    r_off = np.concatenate([[0], np.cumsum(sz)])
    ref = np.array([(d[r_off[i]:r_off[i + 1]] ** 2).sum() for i in range(17)])
    assert np.allclose(row_sq, ref, rtol=1e-13, atol=0)


def test_pattern_digest_sees_one_moved_block():
    m = hamiltonian("sign23", 0, scale=0.1)
    d0 = pattern_digest(m)
    m2 = m.copy()
    # move the last block of a row one column to the right (still canonical)
    i = next(r for r in range(m.nbrows) if m.col_idx[m.row_ptr[r + 1] - 1] < m.nbcols - 1)
    t = int(m2.row_ptr[i + 1]) - 1
    m2.col_idx[t] += 1
    m2.check()
    assert pattern_digest(m2) != d0 and pattern_digest(m.copy()) == d0


@pytest.mark.parametrize("workload,seed", [("sign23", 0), ("sign23", 1), ("sign23", 2),
                                           ("sign23_e5", 0), ("mixed", 0)])
def test_stored_record_is_consistent(workload, seed):
    """A written record belongs to its workload and obeys what the method
    fixes: r_k decreasing to below tol, trace(P) at the occupied count to the
    filter's accuracy, X's block count that of the last iterate."""
    fx = load_fixture(workload, seed)
    if fx is None:
        pytest.skip(f"{fixture_path(workload, seed)} not written")
    w = WORKLOADS[workload]
    assert str(fx["workload"]) == workload and int(fx["seed"]) == seed
    assert float(fx["eps"]) == w["eps"] and float(fx["tol"]) == w["tol"]
    k = int(fx["iterations"])
    r = fx["r_hist"]
    assert r.shape == (k + 1,) and fx["nnzb_x"].shape == (k + 1,) and fx["nnzb_y"].shape == (k + 1,)
    assert r[-1] < w["tol"] and np.all(np.diff(r) < 0)
    assert int(fx["nnzb_final"]) == int(fx["nnzb_x"][-1])
    assert int(fx["n_multiplies"]) == 2 * k + 1
    h = hamiltonian(workload, seed)
    assert h.nbrows == int(fx["sites"])
    assert int(fx["nnzb_x"][0]) == h.nnzb            # X_0 = H / s is not filtered
    assert abs(float(fx["trace_p"]) - h.meta["n_occ"]) < 0.05
    assert fx["xv"].shape == (2, h.shape[0]) and fx["row_sqnorm"].shape == (h.nbrows,)
