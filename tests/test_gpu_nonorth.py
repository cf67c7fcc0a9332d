"""Non-orthogonal basis on the GPU: S^{+-1/2} by the coupled Newton-Schulz
iteration and P = Z (I - sign(Z K Z - mu I)) Z / 2 with Z = S^{-1/2}, each
against the oracle's same steps (block pattern identical, values within the
FP64 tolerance), plus the invariants P S P = P and trace(P S) = occupied
count."""
import numpy as np
import pytest

import synth
from synth import BSR
from tests.gpu_util import TOL_FP64, assert_same_matrix, from_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _opts(eps, tol):
    from paper_2003_03868_amd import bsm
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.max_iter = eps, tol, 100
    return o


@pytest.mark.parametrize("case", [dict(n=100, b=5, rc=4.5, tau=0.4, eps=0.0, seed=7),
                                  dict(n=100, b=5, rc=4.5, tau=0.6, eps=1e-8, seed=8),
                                  dict(n=64, b=13, rc=4.0, tau=0.5, eps=1e-7, seed=9)],
                         ids=lambda c: f"n{c['n']}b{c['b']}t{c['tau']}e{c['eps']:g}")
def test_sqrt_inv_vs_oracle(orc, case):
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(case["n"], case["b"], cutoff=case["rc"], seed=case["seed"])
    s = synth.overlap_like(h, case["tau"], seed=case["seed"])
    sq_ref, isq_ref, st_ref, s_ref = orc.sqrt_inv(s, eps=case["eps"], tol=1e-10)
    d = to_dev(s)
    st, a, b, stats = bsm.bsm_sqrt_inv(d.handle, _opts(case["eps"], 1e-10))
    assert st == s_ref == bsm.OK, bsm.bsm_last_error()
    assert stats.iterations == st_ref["iterations"]
    assert stats.n_multiplies == st_ref["n_multiplies"]
    assert np.allclose(list(stats.r_hist)[:stats.iterations + 1], st_ref["r_hist"], rtol=1e-6,
                       atol=1e-15)
    sz = s.row_blk_size
    assert_same_matrix(from_dev(bsm.Matrix(a, sz, sz)), sq_ref, TOL_FP64, "S^1/2")
    assert_same_matrix(from_dev(bsm.Matrix(b, sz, sz)), isq_ref, TOL_FP64, "S^-1/2")
    print(f"sqrt_inv {case}: {stats.iterations} iterations, {stats.n_multiplies} multiplies")


def test_sqrt_inv_of_identity_stops_at_once(orc):
    """S = 2 I: T_0 = I already, so the iteration stops before any product
    and S^{-1/2} is the diagonal-only I / sqrt(2)."""
    from paper_2003_03868_amd import bsm
    sizes = np.array([3, 5, 2, 4], dtype=np.int32)
    vals = np.concatenate([(2.0 * np.eye(b)).ravel() for b in sizes])
    s = BSR(sizes, sizes, np.arange(5), np.arange(4), vals)
    sq_ref, isq_ref, st_ref, _ = orc.sqrt_inv(s, eps=0.0, tol=1e-12)
    d = to_dev(s)                      # keep the handle alive during the call
    st, a, b, stats = bsm.bsm_sqrt_inv(d.handle, _opts(0.0, 1e-12))
    assert st == bsm.OK and stats.iterations == 0 and stats.n_multiplies == 0
    assert_same_matrix(from_dev(bsm.Matrix(a, sizes, sizes)), sq_ref, 1e-15, "sqrt(2 I)")
    got = from_dev(bsm.Matrix(b, sizes, sizes))
    assert_same_matrix(got, isq_ref, 1e-15, "(2 I)^-1/2")
    assert np.allclose(got.to_dense(), np.eye(int(sizes.sum())) / np.sqrt(2.0), atol=1e-15)


@pytest.mark.parametrize("case", [dict(n=100, b=5, rc=4.5, tau=0.4, eps=1e-8, order=2, seed=7),
                                  dict(n=64, b=13, rc=4.0, tau=0.5, eps=1e-7, order=3, seed=9)],
                         ids=lambda c: f"n{c['n']}b{c['b']}o{c['order']}")
def test_density_nonorth_vs_oracle(orc, case):
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(case["n"], case["b"], cutoff=case["rc"], seed=case["seed"])
    s = synth.overlap_like(h, case["tau"], seed=case["seed"] + 1)
    p_ref, tps_ref, st1_ref, st2_ref, s_ref = orc.density_nonorth(
        h, s, eps=case["eps"], tol=1e-8, order=case["order"])
    o = _opts(case["eps"], 1e-8)
    o.order = case["order"]
    dh, ds = to_dev(h), to_dev(s)      # keep the handles alive during the call
    st, p, tps, st1, st2 = bsm.bsm_density_nonorth(dh.handle, ds.handle, 0.0, o)
    assert st == s_ref == bsm.OK, bsm.bsm_last_error()
    assert st1.iterations == st1_ref["iterations"] and st2.iterations == st2_ref["iterations"]
    sz = h.row_blk_size
    got = from_dev(bsm.Matrix(p, sz, sz))
    assert_same_matrix(got, p_ref, TOL_FP64, "P (non-orthogonal)")
    assert tps == pytest.approx(tps_ref, abs=1e-9)
    assert tps == pytest.approx(h.meta["n_occ"], abs=1e-4)
    pd, sd = got.to_dense(), s.to_dense()
    assert np.linalg.norm(pd @ sd @ pd - pd) / np.linalg.norm(pd) <= 1e-5
    print(f"density_nonorth {case}: sqrt {st1.iterations} it, sign {st2.iterations} it, "
          f"trace(PS) {tps:.8f} (n_occ {h.meta['n_occ']})")


def test_density_nonorth_rejects_mismatched_sizes():
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=1)
    a = synth.random_bsr(10, 10, 5, 5, 0.5, np.random.default_rng(0))
    with pytest.raises(bsm.BsmError) as e:
        dh, da = to_dev(h), to_dev(a)
        bsm.bsm_density_nonorth(dh.handle, da.handle, 0.0)
    assert e.value.status == bsm.EINVAL


def test_failure_modes_report_status(orc):
    """Indefinite S (the coupled iteration cannot converge), TC2 stopped by
    max_iter, a count the bisection cannot reach: each call returns its
    status with the last iterate, as the oracle does."""
    from paper_2003_03868_amd import bsm
    sizes = np.array([2, 3, 2], dtype=np.int32)
    rng = np.random.default_rng(2)
    q, _ = np.linalg.qr(rng.standard_normal((7, 7)))
    d = (q * np.array([-0.5, 0.4, 0.6, 0.8, 1.0, 1.2, 1.4])) @ q.T
    d = 0.5 * (d + d.T)
    off = np.concatenate([[0], np.cumsum(sizes)])
    blocks = [d[off[i]:off[i + 1], off[j]:off[j + 1]].ravel() for i in range(3) for j in range(3)]
    s = BSR(sizes, sizes, np.array([0, 3, 6, 9]), np.tile(np.arange(3), 3), np.concatenate(blocks))
    _, _, st_ref, s_ref = orc.sqrt_inv(s, eps=0.0, tol=1e-12, max_iter=40)
    ds = to_dev(s)
    o = _opts(0.0, 1e-12)
    o.max_iter = 40
    st, a, b, stats = bsm.bsm_sqrt_inv(ds.handle, o)
    assert st == s_ref == bsm.ENOCONV and a and b
    assert stats.iterations == st_ref["iterations"]
    bsm.bsm_destroy(a)
    bsm.bsm_destroy(b)

    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=2)
    dh = to_dev(h)
    o = _opts(0.0, 1e-12)
    o.max_iter = 3
    _, st_ref, s_ref = orc.tc2(h, h.meta["n_occ"], eps=0.0, tol=1e-12, max_iter=3)
    st, ph, stats = bsm.bsm_tc2(dh.handle, h.meta["n_occ"], o)
    assert st == s_ref == bsm.ENOCONV and ph and stats.iterations == 3
    assert list(stats.branch[:3]) == st_ref["branch"]
    bsm.bsm_destroy(ph)

    st, mu, xh, ms = bsm.bsm_mu_bisect(dh.handle, h.meta["n_occ"] + 0.5, -1.0, 1.0,
                                       count_tol=0.1, max_steps=5, opts=_opts(0.0, 1e-10))
    assert st == bsm.ENOCONV and xh and ms.steps == 5
    bsm.bsm_destroy(xh)
