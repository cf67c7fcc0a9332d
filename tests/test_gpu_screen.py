"""Product-level norm screening on the GPU against the oracle's screened
multiply and sign iteration: identical patterns, values within the FP64
tolerance, and the number of left-out products exact."""
import numpy as np
import pytest

import synth
from synth import BSR
from tests.gpu_util import (TOL_FP64, TOL_FP64_MULTIPLY, assert_same_matrix, from_dev, need_gpu,
                            to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _scaled(m: BSR, rng, lo=-4.0) -> BSR:
    off = m.block_offsets()
    v = m.values.copy()
    for t in range(m.nnzb):
        v[off[t]:off[t + 1]] *= 10.0 ** rng.uniform(lo, 0.0)
    return BSR(m.row_blk_size, m.col_blk_size, m.row_ptr, m.col_idx, v)


def _norm_products(a: BSR, b: BSR) -> np.ndarray:
    """Squared-norm products of every block product of A B (host)."""
    sa = np.array([float((a.values[o:e] ** 2).sum()) for o, e in
                   zip(a.block_offsets()[:-1], a.block_offsets()[1:])])
    sb = np.array([float((b.values[o:e] ** 2).sum()) for o, e in
                   zip(b.block_offsets()[:-1], b.block_offsets()[1:])])
    out = []
    for t in range(a.nnzb):
        k = int(a.col_idx[t])
        out.append(sa[t] * sb[b.row_ptr[k]:b.row_ptr[k + 1]])
    return np.concatenate(out) if out else np.zeros(0)


@pytest.mark.parametrize("b", [5, 6, 13, 23, 26, 32])
def test_multiply_screened_vs_oracle(orc, monkeypatch, b):
    from paper_2003_03868_amd import bsm
    rng = np.random.default_rng(800 + b)
    nbr, nbk, nbc = 11, 9, 13
    a = _scaled(synth.random_bsr(nbr, nbk, np.full(nbr, b), np.full(nbk, b), 0.5, rng), rng)
    bm = _scaled(synth.random_bsr(nbk, nbc, np.full(nbk, b), np.full(nbc, b), 0.5, rng), rng)
    c = synth.random_bsr(nbr, nbc, np.full(nbr, b), np.full(nbc, b), 0.3, rng)
    p = np.sort(_norm_products(a, bm))
    # tau^2 in the widest gap around the 40th percentile: no product near the threshold
    lo, hi = int(0.3 * p.size), int(0.5 * p.size)
    g = lo + int(np.argmax(p[lo + 1:hi + 1] / p[lo:hi]))
    tau = float(np.sqrt(np.sqrt(p[g] * p[g + 1])))
    screened = int((p < tau * tau).sum())
    assert 0 < screened < p.size
    for beta, cc in [(0.0, None), (1.5, c)]:
        ref = orc.multiply(-0.7, a, bm, beta, cc, screen=tau)
        da, db = to_dev(a), to_dev(bm)
        dc = to_dev(cc) if cc is not None else bsm.Matrix.empty_like(a.row_blk_size, bm.col_blk_size)
        st = bsm.bsm_multiply_screened(-0.7, da.handle, db.handle, beta, dc.handle, 0.0,
                                       bsm.NORM_FROB, tau)
        got = from_dev(dc)
        assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, f"screened b={b} beta={beta}")
        assert st.n_screened == screened and st.n_products == p.size
        # many chunks and k segments give the same bits
        monkeypatch.setenv("BSM_CHUNK_PRODUCTS", "40")
        monkeypatch.setenv("BSM_TILE_ROWS", "3")
        monkeypatch.setenv("BSM_QUAD_KSEG", "3")
        dc2 = to_dev(cc) if cc is not None else bsm.Matrix.empty_like(a.row_blk_size,
                                                                      bm.col_blk_size)
        st2 = bsm.bsm_multiply_screened(-0.7, da.handle, db.handle, beta, dc2.handle, 0.0,
                                        bsm.NORM_FROB, tau)
        assert np.array_equal(from_dev(dc2).values, got.values)
        assert st2.smm_launches > 1 and st2.n_screened == screened
        for v in ("BSM_CHUNK_PRODUCTS", "BSM_TILE_ROWS", "BSM_QUAD_KSEG"):
            monkeypatch.delenv(v)


def test_screening_zero_is_the_plain_multiply(orc):
    from paper_2003_03868_amd import bsm
    rng = np.random.default_rng(9)
    a = synth.random_bsr(8, 8, np.full(8, 13), np.full(8, 13), 0.5, rng)
    da = to_dev(a)
    c1 = bsm.Matrix.empty_like(a.row_blk_size, a.col_blk_size)
    c2 = bsm.Matrix.empty_like(a.row_blk_size, a.col_blk_size)
    bsm.bsm_multiply(1.0, da.handle, da.handle, 0.0, c1.handle, 0.0)
    st = bsm.bsm_multiply_screened(1.0, da.handle, da.handle, 0.0, c2.handle, 0.0, bsm.NORM_FROB, 0.0)
    assert np.array_equal(from_dev(c1).values, from_dev(c2).values) and st.n_screened == 0


def test_screening_rejects_mixed_sizes_and_bad_thresholds():
    from paper_2003_03868_amd import bsm
    rng = np.random.default_rng(5)
    sz = rng.integers(1, 20, 6)
    a = synth.random_bsr(6, 6, sz, sz, 0.5, rng)
    da = to_dev(a)
    dc = bsm.Matrix.empty_like(sz, sz)
    for tau in (1e-3, -1.0, float("nan")):
        with pytest.raises(bsm.BsmError) as e:
            bsm.bsm_multiply_screened(1.0, da.handle, da.handle, 0.0, dc.handle, 0.0,
                                      bsm.NORM_FROB, tau)
        assert e.value.status == bsm.EINVAL


def test_sign_screened_vs_oracle(orc):
    """The screened Newton-Schulz iteration against the oracle's.  A screening
    decision taken differently (norms summed in another order, within one
    rounding of tau^2) moves one C block by at most tau, far below the
    tolerance here."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(128, 13, cutoff=5.0, seed=7)
    x_ref, st_ref, s_ref = orc.sign_ns(h, eps=1e-7, tol=1e-7, screen=1e-9)
    d = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.eps_screen = 1e-7, 1e-7, 1e-9
    st, xh, stats = bsm.bsm_sign_iterate(d.handle, 0.0, o)
    assert st == s_ref == bsm.OK, bsm.bsm_last_error()
    assert stats.iterations == st_ref["iterations"] and stats.n_screened > 0
    x = bsm.Matrix(xh, h.row_blk_size, h.col_blk_size)
    err = assert_same_matrix(from_dev(x), x_ref, TOL_FP64, "screened sign")
    assert stats.trace_p == pytest.approx(st_ref["trace_p"], abs=1e-6)
    print(f"screened sign: {stats.iterations} iterations, {stats.n_screened} of "
          f"{stats.n_products} products left out, err {err:.2e}")
    x.destroy()
    o.order = 3
    with pytest.raises(bsm.BsmError) as e:
        bsm.bsm_sign_iterate(d.handle, 0.0, o)
    assert e.value.status == bsm.EINVAL
