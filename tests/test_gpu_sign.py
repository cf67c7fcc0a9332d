"""GPU parity of bsm_sign_iterate / bsm_density_from_sign against the CPU
oracle's Newton-Schulz iteration, plus the invariants that hold at any size."""
import numpy as np
import pytest

import synth
from tests.gpu_util import TOL_FP64, assert_same_matrix, from_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _gpu_sign(h, eps=0.0, tol=1e-6, fixed=0, norm="frob", mu=0.0, max_iter=100):
    from paper_2003_03868_amd import bsm
    d = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.fixed_iters, o.max_iter = eps, tol, fixed, max_iter
    o.norm = bsm.NORM_FROB if norm == "frob" else bsm.NORM_MAXABS
    st, xh, stats = bsm.bsm_sign_iterate(d.handle, mu, o)
    x = bsm.Matrix(xh, h.row_blk_size, h.col_blk_size) if xh else None
    return st, x, stats, d


SIGN_CASES = [
    dict(n=64, b=5, rc=4.0, eps=0.0, seed=3),
    dict(n=96, b=13, rc=4.5, eps=0.0, seed=4),
    dict(n=200, b=5, rc=6.0, eps=1e-6, seed=5),
    dict(n=100, b=23, rc=4.2, eps=1e-6, seed=6),
]


@pytest.mark.parametrize("c", SIGN_CASES, ids=lambda c: f"n{c['n']}b{c['b']}e{c['eps']:g}")
def test_sign_vs_oracle(orc, c):
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(c["n"], c["b"], cutoff=c["rc"], seed=c["seed"])
    x_ref, st_ref, s_ref = orc.sign_ns(h, eps=c["eps"], tol=1e-8)
    st, x, stats, _ = _gpu_sign(h, eps=c["eps"], tol=1e-8)
    assert st == bsm.OK and s_ref == orc.OK
    assert stats.iterations == st_ref["iterations"]
    assert np.allclose(list(stats.r_hist)[:stats.iterations + 1], st_ref["r_hist"], rtol=1e-6,
                       atol=1e-15)
    assert stats.scale == pytest.approx(st_ref["scale"], rel=1e-14)
    err = assert_same_matrix(from_dev(x), x_ref, TOL_FP64, "sign")
    assert stats.trace_p == pytest.approx(h.meta["n_occ"], abs=1e-4)
    assert stats.trace_p == pytest.approx(st_ref["trace_p"], abs=1e-9)
    print(f"sign n={c['n']} b={c['b']}: iters {stats.iterations} err {err:.2e}")


def test_sign_fixed_iterations_vs_oracle(orc):
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(128, 13, cutoff=5.0, seed=7)
    x_ref, st_ref, _ = orc.sign_ns(h, eps=1e-5, fixed_iters=4)
    st, x, stats, _ = _gpu_sign(h, eps=1e-5, fixed=4)
    assert st == bsm.OK and stats.iterations == 4
    assert_same_matrix(from_dev(x), x_ref, TOL_FP64, "fixed")


def test_sign_failure_modes(orc):
    from paper_2003_03868_amd import bsm
    sizes = np.array([2, 3], dtype=np.int32)
    # eigenvalue exactly at mu: the residual stalls
    vals = [1.0, 0, 0, -2.0, 0.0, 0, 0, 0, 0, 0, 0, 3.0, 0, 0, 0, 0.5]
    vals = np.array([1.0, 0, 0, -2.0] + [0.0, 0, 0, 0, 3.0, 0, 0, 0, 0.5])
    m = synth.BSR(sizes, sizes, [0, 1, 2], [0, 1], vals)
    st, x, stats, _ = _gpu_sign(m, tol=1e-10)
    assert st == bsm.ENOCONV
    vals2 = vals.copy()
    vals2[4] = np.nan
    st, x, stats, _ = _gpu_sign(synth.BSR(sizes, sizes, [0, 1, 2], [0, 1], vals2), tol=1e-10)
    assert st == bsm.ENONFINITE
    d = to_dev(m)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter = -1.0
    with pytest.raises(bsm.BsmError):
        bsm.bsm_sign_iterate(d.handle, 0.0, o)


def test_density_from_sign(orc):
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=8)
    st, x, stats, _ = _gpu_sign(h, tol=1e-10)
    ph, tp = bsm.bsm_density_from_sign(x.handle)
    p = from_dev(bsm.Matrix(ph, h.row_blk_size, h.col_blk_size))
    ref = orc.density_from_sign(from_dev(x))
    assert_same_matrix(p, ref, 1e-15, "P")
    assert tp == pytest.approx(h.meta["n_occ"], abs=1e-8)
    dp = p.to_dense()
    assert np.linalg.norm(dp @ dp - dp) / dp.shape[0] < 1e-9


def test_sign_mixed_block_sizes_vs_oracle(orc):
    """Neighbour Hamiltonian with block sizes drawn from {5, 13, 23, 26}."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(120, seed=9, cutoff=4.5, size_choices=(5, 13, 23, 26))
    x_ref, st_ref, _ = orc.sign_ns(h, eps=1e-6, tol=1e-8)
    st, x, stats, _ = _gpu_sign(h, eps=1e-6, tol=1e-8)
    assert st == bsm.OK
    assert stats.iterations == st_ref["iterations"]
    assert_same_matrix(from_dev(x), x_ref, TOL_FP64, "mixed sign")
    assert stats.trace_p == pytest.approx(h.meta["n_occ"], abs=1e-4)


@pytest.mark.parametrize("seed", range(6))
def test_add_vs_oracle(orc, seed):
    """bsm_add (C = alpha A + beta B + gamma I, filtered) against the oracle."""
    from paper_2003_03868_amd import bsm
    rng = np.random.default_rng(900 + seed)
    nb = int(rng.integers(1, 12))
    sizes = rng.integers(1, 24, nb)
    a = synth.random_bsr(nb, nb, sizes, sizes, float(rng.choice([0.0, 0.3, 0.8])), rng)
    b = synth.random_bsr(nb, nb, sizes, sizes, float(rng.choice([0.0, 0.3, 0.8])), rng)
    da, db = to_dev(a), to_dev(b)
    alpha, beta = float(rng.normal()), float(rng.normal())
    for gamma in (0.0, 378.0):
        for norm, eps in (("frob", 0.0), ("frob", 0.8), ("maxabs", 0.3)):
            ref = orc.add(alpha, a, beta, b, gamma, eps=eps, norm=norm)
            h = bsm.bsm_add(alpha, da.handle, beta, db.handle, gamma, eps,
                            bsm.NORM_FROB if norm == "frob" else bsm.NORM_MAXABS)
            got = from_dev(bsm.Matrix(h, sizes, sizes))
            assert_same_matrix(got, ref, 1e-14, f"add gamma={gamma} {norm} {eps}")
    h = bsm.bsm_add(-420.0, da.handle, 0.0, None, 315.0)
    assert_same_matrix(from_dev(bsm.Matrix(h, sizes, sizes)), orc.add(-420.0, a, gamma=315.0),
                       1e-14, "add without B")


@pytest.mark.parametrize("order", [3, 5, 7])
@pytest.mark.parametrize("c", [dict(n=64, b=5, rc=4.0, eps=0.0, seed=3),
                               dict(n=200, b=5, rc=6.0, eps=1e-6, seed=5),
                               dict(n=100, b=23, rc=4.2, eps=1e-6, seed=6)],
                         ids=lambda c: f"n{c['n']}b{c['b']}e{c['eps']:g}")
def test_sign_higher_orders_vs_oracle(orc, order, c):
    """Third-, fifth- (Eq. fifth_order_sign: four multiplies per iteration)
    and seventh-order iterations (five multiplies) against the oracle's same
    iterations."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(c["n"], c["b"], cutoff=c["rc"], seed=c["seed"])
    x_ref, st_ref, s_ref = orc.sign_ns(h, eps=c["eps"], tol=1e-8, order=order)
    d = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.order = c["eps"], 1e-8, order
    st, xh, stats = bsm.bsm_sign_iterate(d.handle, 0.0, o)
    assert st == bsm.OK and s_ref == orc.OK, bsm.bsm_last_error()
    assert stats.iterations == st_ref["iterations"]
    assert stats.n_multiplies == st_ref["n_multiplies"]
    assert np.allclose(list(stats.r_hist)[:stats.iterations + 1], st_ref["r_hist"], rtol=1e-6,
                       atol=1e-15)
    x = bsm.Matrix(xh, h.row_blk_size, h.col_blk_size)
    err = assert_same_matrix(from_dev(x), x_ref, TOL_FP64, f"order {order}")
    assert stats.trace_p == pytest.approx(h.meta["n_occ"], abs=1e-4)
    print(f"order {order} n={c['n']} b={c['b']}: iters {stats.iterations}, "
          f"multiplies {stats.n_multiplies}, err {err:.2e}")


def test_mu_bisect_vs_oracle(orc):
    """Chemical-potential bisection for a count inside the unoccupied band:
    the same midpoints and decisions as the oracle's bisection, the accepted
    mu in the eigenvalue gap that gives the count, X at that mu against the
    oracle's."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=3)
    dense = h.to_dense()
    lam = np.linalg.eigvalsh(dense)
    n_occ = h.meta["n_occ"]
    # target: k eigenvalues below mu, k just above n_occ where the gap is widest
    ks = np.arange(n_occ + 1, n_occ + 40)
    k = int(ks[np.argmax(lam[ks] - lam[ks - 1])])
    lo, hi = float(lam[0] - 1.0), float(lam[-1] + 1.0)
    kw = dict(eps=0.0, tol=1e-10, max_iter=100)
    mu_ref, x_ref, rec, s_ref = orc.mu_bisect(h, k, lo, hi, count_tol=0.25, **kw)
    d = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.max_iter = 0.0, 1e-10, 100
    st, mu, xh, stats = bsm.bsm_mu_bisect(d.handle, k, lo, hi, count_tol=0.25, opts=o)
    assert st == s_ref == bsm.OK, bsm.bsm_last_error()
    assert stats.steps == len(rec["mu_hist"])
    assert list(stats.mu_hist[:stats.steps]) == rec["mu_hist"]
    assert np.allclose(list(stats.count_hist[:stats.steps]), rec["count_hist"], atol=1e-7, rtol=0)
    assert mu == mu_ref and int((lam < mu).sum()) == k
    x = bsm.Matrix(xh, h.row_blk_size, h.col_blk_size)
    assert_same_matrix(from_dev(x), x_ref, TOL_FP64, "mu bisection X")
    print(f"mu bisection: k={k}, {stats.steps} steps, mu={mu:.6f}, "
          f"gap [{lam[k - 1]:.6f}, {lam[k]:.6f}], noconv {stats.sign_noconv}")


def test_mu_bisect_rejects_bad_bracket():
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=1)
    d = to_dev(h)
    for lo, hi, steps in [(1.0, -1.0, 10), (0.0, 1.0, 0), (0.0, 1.0, 65)]:
        with pytest.raises(bsm.BsmError) as e:
            bsm.bsm_mu_bisect(d.handle, 10, lo, hi, max_steps=steps)
        assert e.value.status == bsm.EINVAL


@pytest.mark.parametrize("c", [dict(n=100, b=5, rc=4.5, eps=0.0, seed=3),
                               dict(n=100, b=5, rc=4.5, eps=1e-8, seed=4),
                               dict(n=64, b=13, rc=4.0, eps=1e-7, seed=5)],
                         ids=lambda c: f"n{c['n']}b{c['b']}e{c['eps']:g}")
def test_tc2_vs_oracle(orc, c):
    """Trace-correcting purification: the same updates (branch by branch) as
    the oracle, P within the FP64 tolerance, trace(P) the occupied count."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(c["n"], c["b"], cutoff=c["rc"], seed=c["seed"])
    p_ref, st_ref, s_ref = orc.tc2(h, h.meta["n_occ"], eps=c["eps"], tol=1e-9)
    d = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol = c["eps"], 1e-9
    st, ph, stats = bsm.bsm_tc2(d.handle, h.meta["n_occ"], o)
    assert st == s_ref == bsm.OK, bsm.bsm_last_error()
    k = stats.iterations
    assert k == st_ref["iterations"] and list(stats.branch[:k]) == st_ref["branch"]
    assert np.allclose(list(stats.e_hist[:k + 1]), st_ref["e_hist"], rtol=1e-6, atol=1e-14)
    p = bsm.Matrix(ph, h.row_blk_size, h.col_blk_size)
    assert_same_matrix(from_dev(p), p_ref, TOL_FP64, "TC2 P")
    assert stats.trace_p == pytest.approx(h.meta["n_occ"], abs=1e-5)
    print(f"tc2 {c}: {k} iterations, branches {list(stats.branch[:k])}, "
          f"trace(P) {stats.trace_p:.8f}")


@pytest.mark.parametrize("c", [dict(n=100, b=5, rc=4.5, eps=0.0, seed=3),
                               dict(n=100, b=5, rc=4.5, eps=1e-8, seed=4),
                               dict(n=64, b=13, rc=4.0, eps=1e-7, seed=5),
                               dict(n=64, b=23, rc=4.0, eps=1e-9, seed=6)],
                         ids=lambda c: f"n{c['n']}b{c['b']}e{c['eps']:g}")
def test_trs4_vs_oracle(orc, c):
    """Trace-resetting purification: the same updates (branch and gamma) as
    the oracle, P within the FP64 tolerance, trace(P) the occupied count.
    gamma = (N - trace F) / trace G divides two quantities that both vanish
    as X converges: trace F carries a rounding error of about 1e-14 and
    trace G is of the order n e_k^2, so gamma is compared within
    1e-6 |gamma| + 1e-12 / (n e_k^2); X is compared at the end."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(c["n"], c["b"], cutoff=c["rc"], seed=c["seed"])
    p_ref, st_ref, s_ref = orc.trs4(h, h.meta["n_occ"], eps=c["eps"], tol=1e-9)
    d = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol = c["eps"], 1e-9
    st, ph, stats = bsm.bsm_trs4(d.handle, h.meta["n_occ"], o)
    assert st == s_ref == bsm.OK, bsm.bsm_last_error()
    k = stats.iterations
    assert k == st_ref["iterations"] and list(stats.branch[:k]) == st_ref["branch"]
    n = h.shape[0]
    for i in range(k):
        g, gr, e = stats.gamma_hist[i], st_ref["gamma"][i], st_ref["e_hist"][i]
        assert abs(g - gr) <= 1e-6 * abs(gr) + 1e-12 / (n * e * e), (i, g, gr, e)
    assert np.allclose(list(stats.e_hist[:k + 1]), st_ref["e_hist"], rtol=1e-6, atol=1e-14)
    assert stats.n_multiplies == st_ref["n_multiplies"] == 3 * k + 1
    p = bsm.Matrix(ph, h.row_blk_size, h.col_blk_size)
    assert_same_matrix(from_dev(p), p_ref, TOL_FP64, "TRS4 P")
    assert stats.trace_p == pytest.approx(h.meta["n_occ"], abs=1e-5)
    print(f"trs4 {c}: {k} iterations, branches {list(stats.branch[:k])}, "
          f"gamma {[round(g, 3) for g in stats.gamma_hist[:k]]}, trace(P) {stats.trace_p:.8f}")


@pytest.mark.parametrize("frac", [0.9, 0.1])
def test_trs4_out_of_range_updates_vs_oracle(orc, frac):
    """An occupation far from the spectrum's middle: the first updates take
    the TC2 maps (gamma outside [0, 6]); four updates, then ENOCONV, on both
    sides with the same branches and the same X."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=6)
    nocc = round(frac * h.shape[0])
    p_ref, st_ref, s_ref = orc.trs4(h, nocc, eps=0.0, tol=1e-12, max_iter=4)
    d = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.max_iter = 0.0, 1e-12, 4
    st, ph, stats = bsm.bsm_trs4(d.handle, nocc, o)
    assert st == s_ref == bsm.ENOCONV and ph
    assert list(stats.branch[:4]) == st_ref["branch"] and st_ref["branch"][0] in (0, 1)
    p = bsm.Matrix(ph, h.row_blk_size, h.col_blk_size)
    assert_same_matrix(from_dev(p), p_ref, TOL_FP64, "TRS4 X_4")


@pytest.mark.parametrize("full", [False, True], ids=["none", "all"])
def test_degenerate_occupations(full):
    """The degenerate ends of every density-matrix route: mu above (below)
    the whole spectrum, or N = n (N = 0), gives P = I (P = 0).  With a
    filter, P = 0 keeps no block and P = I only the diagonal blocks."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=2)
    n = h.shape[0]
    d = to_dev(h)
    s_inf = float(np.abs(h.to_dense()).sum(1).max())
    mu = 2.0 * s_inf if full else -2.0 * s_inf
    nocc = n if full else 0
    eye = np.eye(n) if full else np.zeros((n, n))
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol = 1e-9, 1e-10

    def check(ph, what):
        p = from_dev(bsm.Matrix(ph, h.row_blk_size, h.col_blk_size))
        assert np.abs(p.to_dense() - eye).max() < 1e-9, what
        assert p.nnzb == (h.nbrows if full else 0), what

    st, xh, stats = bsm.bsm_sign_iterate(d.handle, mu, o)
    assert st == bsm.OK, bsm.bsm_last_error()
    ph, tp = bsm.bsm_density_from_sign(xh)
    bsm.bsm_destroy(xh)
    assert tp == pytest.approx(nocc, abs=1e-9)
    p = from_dev(bsm.Matrix(ph, h.row_blk_size, h.col_blk_size))
    assert np.abs(p.to_dense() - eye).max() < 1e-9
    st, ph, _ = bsm.bsm_submatrix_density(d.handle, mu, o)
    assert st == bsm.OK, bsm.bsm_last_error()
    check(ph, "submatrix")
    for fn in (bsm.bsm_tc2, bsm.bsm_trs4):
        st, ph, stats = fn(d.handle, nocc, o)
        assert st == bsm.OK, bsm.bsm_last_error()
        assert stats.trace_p == pytest.approx(nocc, abs=1e-9)
        check(ph, fn.__name__)
