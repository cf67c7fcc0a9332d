"""The submatrix method on the GPU against the oracle (dense eigendecomposition
per block column): identical patterns, values within the tolerance that the
Newton-Schulz stopping rule leaves (tol 1e-12 on ||X^2 - I||_F / n gives
||X - sign||_F <= n tol / 2), batch splitting bit for bit, failure modes."""
import numpy as np
import pytest

import synth
from synth import BSR
from tests.gpu_util import assert_same_matrix, block_norm_margin, from_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _opts(eps=0.0, tol=1e-12, max_iter=100):
    from paper_2003_03868_amd import bsm
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.max_iter = eps, tol, max_iter
    return o


def _run(h, mu=0.0, **kw):
    from paper_2003_03868_amd import bsm
    d = to_dev(h)
    st, ph, stats = bsm.bsm_submatrix_density(d.handle, mu, _opts(**kw))
    p = bsm.Matrix(ph, h.row_blk_size, h.col_blk_size) if ph else None
    return st, p, stats


CASES = [dict(n=100, b=5, rc=4.5, seed=3, eps=0.0, mu=0.0),
         dict(n=64, b=13, rc=4.0, seed=5, eps=5.8e-3, mu=0.0),
         dict(n=64, b=23, rc=4.0, seed=6, eps=0.0, mu=0.2),
         dict(n=120, b=None, rc=4.5, seed=9, eps=3.07e-3, mu=0.0),
         dict(n=200, b=6, rc=4.0, seed=2, eps=4.277e-3, mu=-0.1)]


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"n{c['n']}b{c['b']}e{c['eps']:g}")
def test_submatrix_vs_oracle(orc, c):
    from paper_2003_03868_amd import bsm
    if c["b"] is None:
        h = synth.neighbour_hamiltonian(c["n"], cutoff=c["rc"], seed=c["seed"],
                                        size_choices=(5, 13, 23, 26))
    else:
        h = synth.neighbour_hamiltonian(c["n"], c["b"], cutoff=c["rc"], seed=c["seed"])
    if c["eps"] > 0:
        raw, _ = orc.submatrix_density(h, mu=c["mu"])
        assert block_norm_margin(raw, c["eps"], "frob").min() > 1e-4
    ref, rec = orc.submatrix_density(h, mu=c["mu"], eps=c["eps"])
    st, p, stats = _run(h, mu=c["mu"], eps=c["eps"])
    assert st == bsm.OK, bsm.bsm_last_error()
    assert stats.n_sub == h.nbrows and stats.max_dim == rec["max_dim"]
    assert stats.r_max < 1e-12 and stats.nnzb == ref.nnzb
    if c["eps"] > 0:
        assert ref.nnzb < h.nnzb
    err = assert_same_matrix(from_dev(p), ref, TOL, f"submatrix {c}")
    print(f"submatrix {c}: {stats.n_sub} submatrices, max dim {stats.max_dim}, mean "
          f"{stats.mean_dim:.0f}, {stats.max_iterations} iterations, err {err:.2e}")


def test_submatrix_batches_give_the_same_bits(monkeypatch):
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(100, 5, cutoff=4.5, seed=4)
    st, p, stats = _run(h)
    assert st == bsm.OK and stats.n_batches == 1
    # about seven submatrices per batch
    monkeypatch.setenv("BSM_SUB_BATCH_BYTES", str(7 * 3 * 8 * 320 * 320))
    st2, p2, stats2 = _run(h)
    assert st2 == bsm.OK and stats2.n_batches > 5
    assert np.array_equal(from_dev(p).values, from_dev(p2).values)


def test_submatrix_full_pattern_is_the_exact_density():
    """Every block stored: each submatrix is the whole matrix, and every
    column comes out of the exact density (LAPACK)."""
    from paper_2003_03868_amd import bsm
    rng = np.random.default_rng(3)
    sizes = np.array([5, 13, 7, 23, 2], dtype=np.int32)
    n = int(sizes.sum())
    a = rng.standard_normal((n, n))
    d = 0.5 * (a + a.T)
    off = np.concatenate([[0], np.cumsum(sizes)])
    vals = [d[off[i]:off[i + 1], off[j]:off[j + 1]].ravel() for i in range(5) for j in range(5)]
    h = BSR(sizes, sizes, np.arange(6) * 5, np.tile(np.arange(5), 5), np.concatenate(vals))
    mu = 0.1
    w, v = np.linalg.eigh(d - mu * np.eye(n))
    ex = v[:, w < 0] @ v[:, w < 0].T
    st, p, stats = _run(h, mu=mu)
    assert st == bsm.OK and stats.max_dim == n
    got = from_dev(p).to_dense()
    assert np.linalg.norm(got - ex) / np.linalg.norm(ex) < TOL


def test_submatrix_failure_modes():
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=1)
    # a block column without its diagonal block
    keep = np.ones(h.nnzb, bool)
    keep[h.row_ptr[3]:h.row_ptr[4]] &= h.col_idx[h.row_ptr[3]:h.row_ptr[4]] != 3
    off = h.block_offsets()
    vals = np.concatenate([h.values[off[t]:off[t + 1]] for t in range(h.nnzb) if keep[t]])
    rp = np.concatenate([[0], np.cumsum([keep[h.row_ptr[i]:h.row_ptr[i + 1]].sum()
                                         for i in range(h.nbrows)])])
    hole = BSR(h.row_blk_size, h.col_blk_size, rp, h.col_idx[keep], vals)
    with pytest.raises(bsm.BsmError) as e:
        _run(hole)
    assert e.value.status == bsm.EINVAL
    # NaN
    bad = BSR(h.row_blk_size, h.col_blk_size, h.row_ptr, h.col_idx, h.values.copy())
    bad.values[7] = np.nan
    st, p, stats = _run(bad)
    assert st == bsm.ENONFINITE and p is None
    # too few iterations: ENOCONV with the last iterates assembled
    st, p, stats = _run(h, max_iter=2)
    assert st == bsm.ENOCONV and p is not None and stats.max_iterations == 2
    for v in (float("nan"), float("inf")):
        with pytest.raises(bsm.BsmError):
            from paper_2003_03868_amd import bsm as b
            d = to_dev(h)
            b.bsm_submatrix_density(d.handle, v, _opts())


def test_submatrix_no_convergence_assembles_every_batch(monkeypatch):
    """Too few iterations: ENOCONV, and the last iterates of every batch are
    assembled (the many-batch result equals the one-batch result bit for
    bit)."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(100, 5, cutoff=4.5, seed=4)
    st, p, stats = _run(h, max_iter=2)
    assert st == bsm.ENOCONV and p is not None and stats.n_batches == 1
    monkeypatch.setenv("BSM_SUB_BATCH_BYTES", str(7 * 3 * 8 * 320 * 320))
    st2, p2, stats2 = _run(h, max_iter=2)
    assert st2 == bsm.ENOCONV and stats2.n_batches > 5
    assert np.array_equal(from_dev(p).values, from_dev(p2).values)
