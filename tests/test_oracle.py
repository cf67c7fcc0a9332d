"""Pins for the CPU oracle: it is checked here against things other than itself
(dense brute force, eigen-decomposition, closed forms, invariants, the
polynomials printed in the paper).  All CPU-only."""
import math
import os

import numpy as np
import pytest

import synth
from synth import BSR

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers

def _rand_case(rng, nbr, nbk, nbc, maxb, dens_a, dens_b, dens_c):
    rs = rng.integers(1, maxb + 1, nbr)
    ks = rng.integers(1, maxb + 1, nbk)
    cs = rng.integers(1, maxb + 1, nbc)
    a = synth.random_bsr(nbr, nbk, rs, ks, dens_a, rng)
    b = synth.random_bsr(nbk, nbc, ks, cs, dens_b, rng)
    c = synth.random_bsr(nbr, nbc, rs, cs, dens_c, rng)
    return a, b, c


def _blocks(m: BSR):
    """dict (i, j) -> dense block, built independently of the oracle."""
    out = {}
    off = 0
    for i in range(m.nbrows):
        for t in range(m.row_ptr[i], m.row_ptr[i + 1]):
            j = int(m.col_idx[t])
            r, c = int(m.row_blk_size[i]), int(m.col_blk_size[j])
            out[(i, j)] = m.values[off:off + r * c].reshape(r, c)
            off += r * c
    return out


def _expected_product(alpha, a, b, beta, c, eps, norm):
    """Dense brute force: D = alpha A B + beta C, pattern by set logic, filter."""
    d = alpha * (a.to_dense() @ b.to_dense())
    if beta != 0.0 and c is not None:
        d = d + beta * c.to_dense()
    pa, pb = a.pattern(), b.pattern()
    rows_of_k = {}
    for (k, j) in pb:
        rows_of_k.setdefault(k, set()).add(j)
    s = set()
    for (i, k) in pa:
        for j in rows_of_k.get(k, ()):
            s.add((i, j))
    if beta != 0.0 and c is not None:
        s |= c.pattern()
    ro = np.concatenate([[0], np.cumsum(a.row_blk_size)])
    co = np.concatenate([[0], np.cumsum(b.col_blk_size)])
    kept, border = {}, 0
    for (i, j) in s:
        blk = d[ro[i]:ro[i + 1], co[j]:co[j + 1]]
        if norm == "frob":
            v, thr = float((blk * blk).sum()), eps * eps
        else:
            v, thr = float(np.abs(blk).max()), eps
        if thr > 0 and abs(v - thr) <= 1e-9 * thr:
            border += 1
        if not (v < thr):
            kept[(i, j)] = blk
    return d, s, kept, border


def _rel(x, y):
    ny = np.linalg.norm(y)
    return np.linalg.norm(x - y) / (ny if ny > 0 else 1.0)


# ---------------------------------------------------------------- multiply

CASES = []
_rng = np.random.default_rng(1234)
for _ in range(40):
    CASES.append(dict(
        nbr=int(_rng.integers(1, 7)), nbk=int(_rng.integers(1, 7)), nbc=int(_rng.integers(1, 7)),
        maxb=int(_rng.choice([1, 5, 13, 32])),
        dens=tuple(float(x) for x in _rng.choice([0.0, 0.3, 0.7, 1.0], 3)),
        alpha=float(_rng.choice([1.0, -0.5, 2.5, 0.0])),
        beta=float(_rng.choice([0.0, 1.0, 1.5, -0.5])),
        eps_q=float(_rng.choice([0.0, 0.3, 0.6])),
        norm=str(_rng.choice(["frob", "maxabs"])),
        seed=int(_rng.integers(0, 2**31)),
    ))


@pytest.mark.parametrize("case", CASES, ids=[f"c{i}" for i in range(len(CASES))])
def test_multiply_matches_dense_bruteforce(orc, case):
    rng = np.random.default_rng(case["seed"])
    a, b, c = _rand_case(rng, case["nbr"], case["nbk"], case["nbc"], case["maxb"], *case["dens"])
    alpha, beta, norm = case["alpha"], case["beta"], case["norm"]
    # choose eps between block norms of the unfiltered product, away from ties
    _, _, unf, _ = _expected_product(alpha, a, b, beta, c, 0.0, norm)
    eps = 0.0
    if case["eps_q"] > 0 and unf:
        if norm == "frob":
            vals = sorted(float(np.sqrt((x * x).sum())) for x in unf.values())
        else:
            vals = sorted(float(np.abs(x).max()) for x in unf.values())
        q = int(case["eps_q"] * (len(vals) - 1))
        eps = vals[q] * 1.0000001 if vals[q] > 0 else 0.0
    d, s, kept, border = _expected_product(alpha, a, b, beta, c, eps, norm)
    assert border == 0
    got = orc.multiply(alpha, a, b, beta, c, eps=eps, norm=norm)
    got.check()
    assert got.pattern() == set(kept.keys())
    gb = _blocks(got)
    for key, blk in kept.items():
        assert _rel(gb[key], blk) <= 1e-13, key


def test_multiply_full_832(orc):
    a, b = synth.random_bsr_pair(64, 13, 0.2, seed=0)
    d, s, kept, _ = _expected_product(1.0, a, b, 0.0, None, 0.0, "frob")
    got = orc.multiply(1.0, a, b)
    assert got.pattern() == s == set(kept.keys())
    assert _rel(got.to_dense(), d) <= 1e-13


def test_multiply_edge_cases(orc):
    rng = np.random.default_rng(7)
    a, b, c = _rand_case(rng, 4, 3, 5, 6, 0.0, 0.5, 0.5)   # empty A
    got = orc.multiply(1.0, a, b)
    assert got.nnzb == 0 and got.values.size == 0
    got = orc.multiply(1.0, a, b, 2.0, c)                   # C = 2 Cin
    assert got.pattern() == c.pattern()
    assert np.array_equal(got.to_dense(), 2.0 * c.to_dense())
    a, b, c = _rand_case(rng, 3, 3, 3, 4, 1.0, 1.0, 0.0)
    got = orc.multiply(0.0, a, b)                           # alpha = 0 keeps the zero blocks
    assert got.nnzb == 9 and not np.any(got.values)
    with pytest.raises(RuntimeError):
        orc.multiply(1.0, a, c if c.nbrows != a.nbcols else
                     synth.random_bsr(3, 3, 9, 9, 1.0, rng))  # block-size mismatch
    with pytest.raises(RuntimeError):
        orc.multiply(1.0, a, b, eps=-1.0)


# ------------------------------------------------------------------ filter

@pytest.mark.parametrize("norm", ["frob", "maxabs"])
def test_filter_rule(orc, norm):
    rng = np.random.default_rng(3)
    m = synth.random_bsr(8, 8, rng.integers(1, 9, 8), rng.integers(1, 9, 8), 0.6, rng)
    m.values *= np.repeat(rng.uniform(0.0, 2.0, m.nnzb) ** 6,
                          np.diff(m.block_offsets()))
    for eps in [0.0, 0.05, 0.5, 3.0]:
        got = orc.filter(m, eps, norm)
        keep = set()
        for key, blk in _blocks(m).items():
            v = float((blk * blk).sum()) if norm == "frob" else float(np.abs(blk).max())
            if not (v < (eps * eps if norm == "frob" else eps)):
                keep.add(key)
        assert got.pattern() == keep
        gb, mb = _blocks(got), _blocks(m)
        for key in keep:
            assert np.array_equal(gb[key], mb[key])


def test_block_sqnorms(orc):
    rng = np.random.default_rng(4)
    m = synth.random_bsr(5, 6, rng.integers(1, 30, 5), rng.integers(1, 30, 6), 0.5, rng)
    ref = [float((blk * blk).sum()) for blk in _blocks(m).values()]
    assert np.allclose(orc.block_sqnorms(m), ref, rtol=1e-14, atol=0)


# ---------------------------------------------------- whole-matrix scalars

def test_scalars_vs_dense(orc):
    rng = np.random.default_rng(5)
    sizes = rng.integers(1, 12, 9)
    m = synth.random_bsr(9, 9, sizes, sizes, 0.4, rng)
    d = m.to_dense()
    n = d.shape[0]
    assert orc.trace(m) == pytest.approx(np.trace(d), rel=1e-14, abs=1e-14)
    for shift in [0.0, 1.0, -2.5]:
        assert orc.sqdist_identity(m, shift) == pytest.approx(
            np.linalg.norm(d - shift * np.eye(n)) ** 2, rel=1e-13)
        assert orc.inf_norm_shifted(m, shift) == pytest.approx(
            np.abs(d - shift * np.eye(n)).sum(1).max(), rel=1e-14)
    sc = orc.shift_scale(m, 0.7, 0.25)
    assert np.allclose(sc.to_dense(), 0.25 * (d - 0.7 * np.eye(n)), rtol=0, atol=1e-15)
    assert all((i, i) in sc.pattern() for i in range(9))


# ---------------------------------------------------------- sign iteration

def _read_polys():
    polys = {}
    with open(os.path.join(GOLDEN, "sign_polynomials.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, order, coef, den = [x.strip() for x in line.split("|")]
            polys[name] = (int(order), [float(x) for x in coef.split()], float(den))
    return polys


def test_golden_polynomials_are_sign_iterations():
    """Closed form: g(x) = x q(x^2)/den has g(1) = 1 and g'(x) = c (1-x^2)^(p-1)."""
    for name, (order, coef, den) in _read_polys().items():
        # g(x) as a polynomial in x
        g = np.zeros(2 * len(coef))
        for p, cf in enumerate(coef):
            g[2 * p + 1] = cf / den
        gp = np.polynomial.polynomial.polyder(g)
        target = np.polynomial.polynomial.polypow([1.0, 0.0, -1.0], order - 1)
        ratio = gp[0] / target[0]
        assert np.allclose(gp, ratio * target[:gp.size], atol=1e-12), name
        assert np.polynomial.polynomial.polyval(1.0, g) == pytest.approx(1.0, abs=1e-14)
        assert ratio > 0


def _diag_matrix(vals, sizes):
    """Block-diagonal BSR whose blocks are diagonal matrices."""
    sizes = np.asarray(sizes, dtype=np.int32)
    nb = sizes.size
    blocks, p = [], 0
    for s in sizes:
        blk = np.zeros((s, s))
        blk[np.arange(s), np.arange(s)] = vals[p:p + s]
        p += s
        blocks.append(blk.ravel())
    return BSR(sizes, sizes, np.arange(nb + 1), np.arange(nb), np.concatenate(blocks))


def test_sign_diagonal_scalar_recurrence(orc):
    """Diagonal H: the iteration decouples into the scalar f_1 recurrence,
    evaluated here in the same operation order, so X must agree bit for bit."""
    rng = np.random.default_rng(11)
    sizes = rng.integers(1, 7, 10)
    n = int(sizes.sum())
    h = rng.uniform(0.05, 5.0, n) * rng.choice([-1.0, 1.0], n)
    mu = 0.01
    tol = 1e-9
    m = _diag_matrix(h, sizes)
    x_got, st, status = orc.sign_ns(m, mu=mu, eps=0.0, tol=tol)
    assert status == orc.OK
    x = (h - mu) * (1.0 / np.abs(h - mu).max())
    rs = []
    for k in range(100):
        y = x * x
        r = math.sqrt(float(((y - 1.0) ** 2).sum())) / n
        rs.append(r)
        if r < tol:
            break
        x = -0.5 * (x * y) + 1.5 * x
    assert st["iterations"] == k
    assert np.allclose(st["r_hist"], rs, rtol=1e-13, atol=0)
    assert np.array_equal(np.diag(x_got.to_dense()), x)
    # same result through the printed polynomial f_1 = x (3 - x^2)/2
    order, coef, den = _read_polys()["f1"]
    xp = (h - mu) * (1.0 / np.abs(h - mu).max())
    for _ in range(k):
        y = xp * xp
        xp = xp * (coef[0] + coef[1] * y) / den
    assert np.allclose(xp, x, rtol=0, atol=1e-14)
    assert st["trace_p"] == pytest.approx(0.5 * (n - x.sum()), abs=1e-12)


def _eig_sign(d, mu=0.0):
    w, v = np.linalg.eigh(d - mu * np.eye(d.shape[0]))
    return (v * np.sign(w)) @ v.T, int((w < 0).sum())


def _dense_to_bsr(d, sizes, keep_frac=1.0, rng=None):
    sizes = np.asarray(sizes, dtype=np.int32)
    off = np.concatenate([[0], np.cumsum(sizes)])
    nb = sizes.size
    rp, ci, vals = [0], [], []
    for i in range(nb):
        for j in range(nb):
            blk = d[off[i]:off[i + 1], off[j]:off[j + 1]]
            if np.any(blk):
                ci.append(j)
                vals.append(blk.ravel())
        rp.append(len(ci))
    return BSR(sizes, sizes, np.array(rp), np.array(ci), np.concatenate(vals))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_sign_matches_eigh_dense(orc, seed):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 14, 8)
    n = int(sizes.sum())
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(0.1, 3.0, n) * rng.choice([-1.0, 1.0], n)
    d = (q * lam) @ q.T
    d = 0.5 * (d + d.T)
    m = _dense_to_bsr(d, sizes)
    x, st, status = orc.sign_ns(m, mu=0.0, eps=0.0, tol=1e-13)
    assert status == orc.OK
    ref, nneg = _eig_sign(d)
    dx = x.to_dense()
    assert _rel(dx, ref) <= 1e-12
    assert np.linalg.norm(dx - dx.T) / np.linalg.norm(dx) < 1e-12
    assert st["trace_p"] == pytest.approx(nneg, abs=1e-9)


def test_sign_2x2_closed_form(orc):
    """sign(M) = (2M - tr(M) I)/sqrt(tr^2 - 4 det) when det < 0, else +-I."""
    rng = np.random.default_rng(9)
    for _ in range(20):
        a, b, c = rng.normal(size=3) * 3
        mm = np.array([[a, b], [b, c]])
        tr, det = a + c, a * c - b * b
        if abs(det) < 1e-3:
            continue
        ref = (2 * mm - tr * np.eye(2)) / math.sqrt(tr * tr - 4 * det) if det < 0 \
            else np.sign(tr) * np.eye(2)
        for sizes in ([2], [1, 1]):
            x, st, status = orc.sign_ns(_dense_to_bsr(mm, sizes), tol=1e-14)
            assert status == orc.OK
            assert np.allclose(x.to_dense(), ref, rtol=0, atol=1e-13)


def test_sign_neighbour_hamiltonian_vs_eigh(orc):
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=3)
    x, st, status = orc.sign_ns(h, eps=0.0, tol=1e-12)
    assert status == orc.OK
    ref, nneg = _eig_sign(h.to_dense())
    assert nneg == h.meta["n_occ"]
    assert _rel(x.to_dense(), ref) <= 1e-11
    assert st["trace_p"] == pytest.approx(h.meta["n_occ"], abs=1e-8)


def test_sign_block_diagonal_vs_eigh(orc):
    """Cutoff below every pair distance: each diagonal block on its own."""
    h = synth.neighbour_hamiltonian(40, 7, cutoff=0.05, seed=2)
    assert h.meta["n_pairs"] == 0
    x, st, status = orc.sign_ns(h, eps=0.0, tol=1e-13)
    assert status == orc.OK
    xb = _blocks(x)
    for (i, j), blk in _blocks(h).items():
        ref, _ = _eig_sign(blk)
        assert np.allclose(xb[(i, j)], ref, rtol=0, atol=1e-12)


def test_sign_with_filter_invariants(orc):
    h = synth.neighbour_hamiltonian(200, 5, cutoff=6.0, seed=4)
    tol = 1e-7
    x, st, status = orc.sign_ns(h, eps=1e-6, tol=tol)
    assert status == orc.OK
    n = h.shape[0]
    d = x.to_dense()
    # X Y and Y X differ once Y is filtered, so symmetry only holds to O(eps)
    assert np.linalg.norm(d - d.T) / np.linalg.norm(d) < 1e-5
    assert np.linalg.norm(d @ d - np.eye(n)) / n < 10 * tol
    assert st["trace_p"] == pytest.approx(h.meta["n_occ"], abs=1e-3)
    ref, _ = _eig_sign(h.to_dense())
    assert _rel(d, ref) < 1e-4
    # a coarse filter drops blocks, and r_k (taken on the filtered square)
    # still reaches tol while the exact residual stays at the filter's level
    x, st, status = orc.sign_ns(h, eps=1e-3, tol=1e-5)
    assert status == orc.OK and x.nnzb < h.nbrows ** 2
    d = x.to_dense()
    assert np.linalg.norm(d @ d - np.eye(n)) / n < 1e-3
    assert st["trace_p"] == pytest.approx(h.meta["n_occ"], abs=1e-2)


def test_sign_fixed_iters(orc):
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=5)
    x3, st3, s3 = orc.sign_ns(h, fixed_iters=3)
    assert s3 == orc.OK and st3["iterations"] == 3 and len(st3["r_hist"]) == 4
    x, st, s = orc.sign_ns(h, tol=0.0, max_iter=3)
    assert s == orc.ENOCONV
    assert np.array_equal(x.values, x3.values)


def test_sign_failure_modes(orc):
    sizes = np.array([2, 3])
    vals = np.array([1.0, -2.0, 0.0, 3.0, 0.5])       # an eigenvalue exactly at mu = 0
    x, st, status = orc.sign_ns(_diag_matrix(vals, sizes), tol=1e-10)
    assert status == orc.ENOCONV
    vals = np.array([1.0, -2.0, np.nan, 3.0, 0.5])
    x, st, status = orc.sign_ns(_diag_matrix(vals, sizes), tol=1e-10)
    assert status == orc.ENONFINITE


def test_density_matrix_identities(orc):
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=6)
    x, st, _ = orc.sign_ns(h, tol=1e-8)
    p = orc.density_from_sign(x)
    n = h.shape[0]
    dp, dx = p.to_dense(), x.to_dense()
    assert np.allclose(dp, 0.5 * (np.eye(n) - dx), rtol=0, atol=1e-15)
    lhs = np.linalg.norm(dp @ dp - dp)
    assert lhs == pytest.approx(0.25 * np.linalg.norm(dx @ dx - np.eye(n)), rel=1e-6)
    assert orc.trace(p) == pytest.approx(st["trace_p"], abs=1e-12)


# ----------------------------------------------------------- matrix sum

def _expected_add(alpha, a, beta, b, gamma, eps, norm):
    """Dense alpha A + beta B + gamma I, pattern by set logic, then the filter."""
    d = alpha * a.to_dense()
    s = set(a.pattern())
    if b is not None:
        d = d + beta * b.to_dense()
        s |= b.pattern()
    if gamma != 0.0:
        d = d + gamma * np.eye(d.shape[0])
        s |= {(i, i) for i in range(a.nbrows)}
    ro = np.concatenate([[0], np.cumsum(a.row_blk_size)])
    co = np.concatenate([[0], np.cumsum(a.col_blk_size)])
    kept = {}
    for (i, j) in s:
        blk = d[ro[i]:ro[i + 1], co[j]:co[j + 1]]
        v, thr = ((float((blk * blk).sum()), eps * eps) if norm == "frob"
                  else (float(np.abs(blk).max()), eps))
        if not (v < thr):
            kept[(i, j)] = blk
    return kept


@pytest.mark.parametrize("seed", range(8))
def test_add_matches_dense(orc, seed):
    """C = alpha A + beta B + gamma I against dense arithmetic and set logic."""
    rng = np.random.default_rng(700 + seed)
    nb = int(rng.integers(1, 9))
    sizes = rng.integers(1, 12, nb)
    a = synth.random_bsr(nb, nb, sizes, sizes, float(rng.choice([0.0, 0.3, 0.7])), rng)
    b = synth.random_bsr(nb, nb, sizes, sizes, float(rng.choice([0.0, 0.3, 0.7])), rng)
    alpha, beta = float(rng.normal()), float(rng.normal())
    for gamma in (0.0, 378.0):
        for norm, eps in (("frob", 0.0), ("frob", 0.8), ("maxabs", 0.3)):
            got = orc.add(alpha, a, beta, b, gamma, eps=eps, norm=norm)
            exp = _expected_add(alpha, a, beta, b, gamma, eps, norm)
            gb = _blocks(got)
            assert set(gb) == set(exp)
            for key, blk in exp.items():
                assert np.allclose(gb[key], blk, rtol=1e-15, atol=1e-15)
    # B absent
    got = orc.add(-420.0, a, gamma=315.0)
    assert set(_blocks(got)) == set(_expected_add(-420.0, a, 0.0, None, 315.0, 0.0, "frob"))


# ------------------------------------------- higher-order sign iterations

def _family_poly(order):
    """q of the order-p member of the family the printed polynomials belong
    to (g'(x) proportional to (1 - x^2)^(p-1), g(0) = 0, g(1) = 1, g(x) =
    x q(x^2)), by integrating the closed form with numpy: the paper names
    the seventh-order iteration without printing it."""
    P = np.polynomial.polynomial
    g = P.polyint(P.polypow([1.0, 0.0, -1.0], order - 1))
    g = g / P.polyval(1.0, g)
    return list(g[1::2]), 1.0


@pytest.mark.parametrize("order,poly", [(2, "f1"), (3, "f2"), (5, "p5"), (7, None)])
def test_sign_orders_follow_printed_polynomials(orc, order, poly):
    """Diagonal H: every update of the order-p iteration must equal the
    polynomial printed in the paper (OT/IR f_1, f_2; Eq. fifth_order_sign)
    or, for order 7, the family member derived from its closed form,
    g(x) = x q(x^2)/den, evaluated independently with numpy."""
    coef, den = _family_poly(order) if poly is None else _read_polys()[poly][1:]
    rng = np.random.default_rng(40 + order)
    sizes = rng.integers(1, 6, 9)
    n = int(sizes.sum())
    h = rng.uniform(0.05, 4.0, n) * rng.choice([-1.0, 1.0], n)
    m = _diag_matrix(h, sizes)
    x = h / np.abs(h).max()
    for k in range(1, 4):
        xk, st, status = orc.sign_ns(m, eps=0.0, fixed_iters=k, order=order)
        assert status == orc.OK and st["iterations"] == k
        x = x * np.polynomial.polynomial.polyval(x * x, coef) / den
        assert np.allclose(np.diag(xk.to_dense()), x, rtol=1e-13, atol=1e-15)
        per_update = {2: 2, 3: 3, 5: 4, 7: 5}[order]
        assert st["n_multiplies"] == per_update * k + 1


@pytest.mark.parametrize("order", [3, 5, 7])
@pytest.mark.parametrize("seed", [0, 1])
def test_sign_higher_orders_match_eigh(orc, order, seed):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 14, 8)
    n = int(sizes.sum())
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(0.1, 3.0, n) * rng.choice([-1.0, 1.0], n)
    d = (q * lam) @ q.T
    d = 0.5 * (d + d.T)
    m = _dense_to_bsr(d, sizes)
    x, st, status = orc.sign_ns(m, eps=0.0, tol=1e-13, order=order)
    assert status == orc.OK
    _, st2, _ = orc.sign_ns(m, eps=0.0, tol=1e-13, order=2)
    assert st["iterations"] < st2["iterations"]
    ref, nneg = _eig_sign(d)
    assert _rel(x.to_dense(), ref) <= 1e-12
    assert st["trace_p"] == pytest.approx(nneg, abs=1e-9)


def test_sign_higher_orders_filtered_neighbour(orc):
    """Filtered order-5 run on a neighbour Hamiltonian: trace(P) is the
    occupied count and X^2 is the identity to the filter's accuracy."""
    h = synth.neighbour_hamiltonian(200, 5, cutoff=6.0, seed=4)
    x, st, status = orc.sign_ns(h, eps=1e-6, tol=1e-7, order=5)
    assert status == orc.OK
    assert st["trace_p"] == pytest.approx(h.meta["n_occ"], abs=1e-4)
    dx = x.to_dense()
    assert np.linalg.norm(dx @ dx - np.eye(dx.shape[0])) / dx.shape[0] < 1e-5


# ------------------------------------------------ chemical potential search

def test_mu_bisect_diagonal_by_hand(orc):
    """Diagonal H: count(mu) is the number of diagonal entries below mu, so
    the bisection's midpoints and decisions follow by hand exactly."""
    rng = np.random.default_rng(21)
    sizes = rng.integers(1, 6, 12)
    n = int(sizes.sum())
    h = rng.uniform(-4.0, 4.0, n)
    m = _diag_matrix(h, sizes)
    target = n // 3
    mu, x, rec, status = orc.mu_bisect(m, target, -5.0, 5.0, count_tol=0.25, max_steps=40,
                                       eps=0.0, tol=1e-12)
    assert status == orc.OK
    lo, hi, hand = -5.0, 5.0, []
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        c = int((h < mid).sum())
        hand.append((mid, c))
        if abs(c - target) <= 0.25:
            break
        if c < target:
            lo = mid
        else:
            hi = mid
    assert rec["mu_hist"] == [a for a, _ in hand]
    assert np.allclose(rec["count_hist"], [c for _, c in hand], atol=1e-8, rtol=0)
    assert mu == hand[-1][0] and int((h < mu).sum()) == target
    # the returned X is sign(H - mu I)
    assert np.allclose(np.diag(x.to_dense()), np.sign(h - mu), atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1])
def test_mu_bisect_dense_lands_in_gap(orc, seed):
    rng = np.random.default_rng(60 + seed)
    sizes = rng.integers(2, 9, 8)
    n = int(sizes.sum())
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.sort(rng.uniform(-3.0, 3.0, n))
    d = (q * lam) @ q.T
    d = 0.5 * (d + d.T)
    m = _dense_to_bsr(d, sizes)
    gaps = np.diff(lam)
    k = int(np.argmax(gaps[n // 4:3 * n // 4])) + n // 4 + 1    # k eigenvalues below the gap
    mu, x, rec, status = orc.mu_bisect(m, k, lam[0] - 1.0, lam[-1] + 1.0, count_tol=0.25,
                                       eps=0.0, tol=1e-12)
    assert status == orc.OK
    w = np.linalg.eigvalsh(d)
    assert int((w < mu).sum()) == k
    assert rec["count_hist"][-1] == pytest.approx(k, abs=1e-8)
    ref, _ = _eig_sign(d - mu * np.eye(n))
    assert _rel(x.to_dense(), ref) <= 1e-11


def test_mu_bisect_reports_no_convergence(orc):
    """A target no midpoint can reach within count_tol (half-integer with a
    tight tolerance) ends with ENOCONV after max_steps, with the last mu."""
    h = np.array([-1.0, 1.0, 2.0])
    m = _diag_matrix(h, [1, 1, 1])
    mu, x, rec, status = orc.mu_bisect(m, 1.5, -3.0, 3.0, count_tol=0.1, max_steps=6,
                                       eps=0.0, tol=1e-12)
    assert status == orc.ENOCONV and len(rec["mu_hist"]) == 6 and x is not None


# --------------------------------------------- non-orthogonal basis (S != I)

def _spd(rng, n, lo=0.3, hi=2.0):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = (q * rng.uniform(lo, hi, n)) @ q.T
    return 0.5 * (d + d.T)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sqrt_inv_matches_eigh(orc, seed):
    """Coupled iteration on tiny dense SPD matrices: S^{1/2} and S^{-1/2}
    against the eigen-decomposition (LAPACK)."""
    rng = np.random.default_rng(80 + seed)
    sizes = rng.integers(1, 9, 7)
    n = int(sizes.sum())
    d = _spd(rng, n)
    w, v = np.linalg.eigh(d)
    ref_sqrt = (v * np.sqrt(w)) @ v.T
    ref_isqrt = (v / np.sqrt(w)) @ v.T
    sq, isq, st, status = orc.sqrt_inv(_dense_to_bsr(d, sizes), eps=0.0, tol=1e-14)
    assert status == orc.OK
    assert _rel(sq.to_dense(), ref_sqrt) <= 1e-12
    assert _rel(isq.to_dense(), ref_isqrt) <= 1e-12
    assert st["n_multiplies"] == 3 * st["iterations"] - 1


def test_sqrt_inv_diagonal_by_hand(orc):
    """Diagonal S: the coupled iteration decouples into the scalar
    recurrence y <- y w, z <- w z, w = -0.5 (z y - 3), from y = s/||S||_inf,
    z = 1 (first step: t = y, z_1 = w), evaluated here in the same order."""
    rng = np.random.default_rng(31)
    sizes = rng.integers(1, 6, 9)
    sv = rng.uniform(0.2, 3.0, int(sizes.sum()))
    n = sv.size
    m = _diag_matrix(sv, sizes)
    sq, isq, st, status = orc.sqrt_inv(m, eps=0.0, tol=1e-13)
    assert status == orc.OK
    sc = sv.max()
    y = sv * (1.0 / sc)
    z = None
    rs = []
    for k in range(100):
        t = y if z is None else z * y
        rs.append(math.sqrt(float(((t - 1.0) ** 2).sum())) / n)
        if rs[-1] < 1e-13:
            break
        w = -0.5 * (t - 3.0)
        y, z = y * w, (w if z is None else w * z)
    assert st["iterations"] == k
    assert np.allclose(st["r_hist"], rs, rtol=1e-12, atol=0)
    assert np.array_equal(np.diag(sq.to_dense()), math.sqrt(sc) * (y - 0.0))
    assert np.array_equal(np.diag(isq.to_dense()), (1.0 / math.sqrt(sc)) * (z - 0.0))


@pytest.mark.parametrize("seed", [0, 1])
def test_density_nonorth_matches_generalised_eigh(orc, seed):
    """P = (I - sign(S^{-1} K - mu I)) S^{-1} / 2 equals C_occ C_occ^T for the
    S-orthonormal eigenvectors of K c = e S c with e < mu (LAPACK), and
    trace(P S) is their number."""
    import scipy.linalg
    rng = np.random.default_rng(90 + seed)
    sizes = rng.integers(1, 8, 7)
    n = int(sizes.sum())
    s = _spd(rng, n, 0.5, 1.5)
    kq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    k = (kq * (rng.uniform(0.2, 2.0, n) * rng.choice([-1.0, 1.0], n))) @ kq.T
    k = 0.5 * (k + k.T)
    mu = 0.05
    e, c = scipy.linalg.eigh(k, s)
    occ = c[:, e < mu]
    p_ref = occ @ occ.T
    p, tps, st1, st2, status = orc.density_nonorth(_dense_to_bsr(k, sizes), _dense_to_bsr(s, sizes),
                                                   mu=mu, eps=0.0, tol=1e-13)
    assert status == orc.OK
    assert _rel(p.to_dense(), p_ref) <= 1e-10
    assert tps == pytest.approx(int((e < mu).sum()), abs=1e-9)
    pd = p.to_dense()
    assert _rel(pd @ s @ pd, pd) <= 1e-10


def test_density_nonorth_neighbour_invariants(orc):
    """Filtered run on a neighbour Hamiltonian with a decaying overlap: the
    occupied count is the inertia of K (Sylvester: Z K Z is congruent to K),
    and P S P = P to the filter's accuracy."""
    h = synth.neighbour_hamiltonian(100, 5, cutoff=4.5, seed=7)
    s = synth.overlap_like(h, 0.4, seed=2)
    p, tps, st1, st2, status = orc.density_nonorth(h, s, eps=1e-8, tol=1e-8)
    assert status == orc.OK
    assert tps == pytest.approx(h.meta["n_occ"], abs=1e-4)
    pd, sd = p.to_dense(), s.to_dense()
    assert _rel(pd @ sd @ pd, pd) <= 1e-5
    assert float(np.trace(pd @ sd)) == pytest.approx(h.meta["n_occ"], abs=1e-3)


# --------------------------------------- trace-correcting purification (TC2)

def test_tc2_diagonal_by_hand(orc):
    """Diagonal H: X stays diagonal, so every update is the scalar map x^2 or
    2x - x^2 chosen by the trace against N, evaluated here in the same order."""
    rng = np.random.default_rng(41)
    sizes = rng.integers(1, 6, 10)
    h = rng.uniform(-3.0, 3.0, int(sizes.sum()))
    n = h.size
    nocc = int((h < 0.2).sum())
    m = _diag_matrix(h, sizes)
    p, st, status = orc.tc2(m, nocc, eps=0.0, tol=1e-13)
    assert status == orc.OK
    s = np.abs(h).max()
    x = -(0.5 / s) * (h - s)
    branches, es = [], []
    for k in range(100):
        y = x * x
        e = (x.sum() - y.sum()) / n
        es.append(e)
        if e < 1e-13:
            break
        if x.sum() > nocc:
            branches.append(0)
            x = y
        else:
            branches.append(1)
            x = 2.0 * x + (-1.0) * y
    assert st["iterations"] == k and st["branch"] == branches
    assert np.allclose(st["e_hist"], es, rtol=1e-10, atol=1e-16)
    assert np.array_equal(np.diag(p.to_dense()), x)
    assert np.array_equal(np.round(x), (h < np.sort(h)[nocc - 1] + 1e-12).astype(float))


@pytest.mark.parametrize("seed", [0, 1])
def test_tc2_dense_is_the_occupied_projector(orc, seed):
    rng = np.random.default_rng(70 + seed)
    sizes = rng.integers(1, 9, 8)
    n = int(sizes.sum())
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.sort(rng.uniform(-2.0, 2.0, n))
    nocc = n // 3
    lam[nocc:] += 0.5                         # a gap above the N-th eigenvalue
    d = (q * lam) @ q.T
    d = 0.5 * (d + d.T)
    p, st, status = orc.tc2(_dense_to_bsr(d, sizes), nocc, eps=0.0, tol=1e-14)
    assert status == orc.OK
    w, v = np.linalg.eigh(d)
    ref = v[:, :nocc] @ v[:, :nocc].T
    assert _rel(p.to_dense(), ref) <= 1e-10
    assert st["trace_p"] == pytest.approx(nocc, abs=1e-9)


def test_tc2_matches_sign_density_on_neighbour_hamiltonian(orc):
    """With the gap of the synthetic Hamiltonian, the canonical TC2 density
    for N = the occupied count and the sign-iteration density at mu = 0 are
    the same projector, up to the filter."""
    h = synth.neighbour_hamiltonian(100, 5, cutoff=4.5, seed=3)
    p, st, status = orc.tc2(h, h.meta["n_occ"], eps=1e-9, tol=1e-9)
    assert status == orc.OK
    x, _, s2 = orc.sign_ns(h, eps=1e-9, tol=1e-9)
    ps = orc.density_from_sign(x)
    assert _rel(p.to_dense(), ps.to_dense()) <= 1e-6
    assert st["trace_p"] == pytest.approx(h.meta["n_occ"], abs=1e-5)


# ---------------------------------------------------------------- transpose

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_transpose_is_the_dense_transpose(orc, seed):
    rng = np.random.default_rng(300 + seed)
    nbr, nbc = int(rng.integers(1, 9)), int(rng.integers(1, 9))
    a = synth.random_bsr(nbr, nbc, rng.integers(1, 33, nbr), rng.integers(1, 33, nbc), 0.4, rng)
    t = orc.transpose(a)
    t.check()
    assert np.array_equal(t.row_blk_size, a.col_blk_size)
    assert np.array_equal(t.to_dense(), a.to_dense().T)
    back = orc.transpose(t)
    for f in ("row_ptr", "col_idx", "values"):
        assert np.array_equal(getattr(back, f), getattr(a, f))


# ------------------------------------ trace-resetting purification (TRS4)

def _trs4_diag_case(seed, nocc_frac):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 6, 12)
    h = rng.uniform(-3.0, 3.0, int(sizes.sum()))
    h[0], h[1] = 3.5, -3.5                     # entries that start at exactly 0 and 1
    return h, sizes, int(round(nocc_frac * h.size))


@pytest.mark.parametrize("frac", [0.45, 0.6])
def test_trs4_one_update_is_a_fourth_order_map_with_the_trace_reset(orc, frac):
    """Diagonal H, one update: every entry moves by the same quartic p with
    p(0) = 0, p'(0) = 0, p(1) = 1, p'(1) = 0 (the conditions that make the
    purification fourth-order at both fixed points), and the trace lands on
    N.  p is fitted here from the data, not taken from the oracle's formula:
    x1 / x0^2 = a + b x0 + c x0^2 must hold for every entry, with
    a + b + c = 1 (p(1) = 1) and b + 2c = -2 (p'(1) = 0)."""
    h, sizes, nocc = _trs4_diag_case(43, frac)
    p, st, status = orc.trs4(_diag_matrix(h, sizes), nocc, eps=0.0, tol=1e-15, max_iter=1)
    assert status == orc.ENOCONV and st["branch"] == [2]
    s = np.abs(h).max()
    x0 = -(0.5 / s) * (h - s)
    x1 = np.diag(p.to_dense())
    assert x0[0] == 0.0 and x0[1] == 1.0 and x1[0] == 0.0 and x1[1] == pytest.approx(1.0, abs=1e-15)
    sel = x0 > 0.05
    a, b, c = np.linalg.lstsq(np.stack([np.ones(sel.sum()), x0[sel], x0[sel] ** 2], 1),
                              x1[sel] / x0[sel] ** 2, rcond=None)[0]
    assert np.allclose(x1, x0 ** 2 * (a + b * x0 + c * x0 ** 2), rtol=0, atol=1e-13)
    assert a + b + c == pytest.approx(1.0, abs=1e-11)
    assert b + 2 * c == pytest.approx(-2.0, abs=1e-11)
    assert x1.sum() == pytest.approx(nocc, abs=1e-11)
    # the family's free coefficient is gamma - 3 in the x^4 term
    assert st["gamma"][0] == pytest.approx(c + 3.0, abs=1e-10) and 0.0 <= st["gamma"][0] <= 6.0


@pytest.mark.parametrize("seed,frac,branch", [(44, 0.98, 1), (44, 0.02, 0), (43, 0.65, 1),
                                               (43, 0.4, 0)])
def test_trs4_out_of_range_updates_by_hand(orc, seed, frac, branch):
    """An occupation no member of the family can reach (gamma outside
    [0, 6]) takes the TC2 map that moves the trace the right way:
    2x - x^2 to raise it, x^2 to lower it (the last two cases lie just
    outside the range: gamma 6.4 and -0.6)."""
    h, sizes, nocc = _trs4_diag_case(seed, frac)
    p, st, status = orc.trs4(_diag_matrix(h, sizes), nocc, eps=0.0, tol=1e-15, max_iter=1)
    assert status == orc.ENOCONV and st["branch"] == [branch]
    assert (st["gamma"][0] > 6.0) if branch == 1 else (st["gamma"][0] < 0.0)
    s = np.abs(h).max()
    x0 = -(0.5 / s) * (h - s)
    want = 2.0 * x0 + (-1.0) * (x0 * x0) if branch == 1 else x0 * x0
    assert np.array_equal(np.diag(p.to_dense()), want)


def test_trs4_diagonal_converges_to_the_occupied_set(orc):
    h, sizes, nocc = _trs4_diag_case(45, 0.4)
    p, st, status = orc.trs4(_diag_matrix(h, sizes), nocc, eps=0.0, tol=1e-13)
    assert status == orc.OK
    x = np.diag(p.to_dense())
    assert np.allclose(x, (h <= np.sort(h)[nocc - 1]).astype(float), atol=1e-6)
    assert st["n_multiplies"] == 3 * st["iterations"] + 1


@pytest.mark.parametrize("seed", [0, 1])
def test_trs4_dense_is_the_occupied_projector(orc, seed):
    rng = np.random.default_rng(90 + seed)
    sizes = rng.integers(1, 9, 8)
    n = int(sizes.sum())
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.sort(rng.uniform(-2.0, 2.0, n))
    nocc = n // 3 + seed
    lam[nocc:] += 0.5
    d = (q * lam) @ q.T
    d = 0.5 * (d + d.T)
    p, st, status = orc.trs4(_dense_to_bsr(d, sizes), nocc, eps=0.0, tol=1e-14)
    assert status == orc.OK
    w, v = np.linalg.eigh(d)
    ref = v[:, :nocc] @ v[:, :nocc].T
    assert _rel(p.to_dense(), ref) <= 1e-10
    assert st["trace_p"] == pytest.approx(nocc, abs=1e-9)
    assert 2 in st["branch"]


def test_trs4_matches_tc2_on_neighbour_hamiltonian(orc):
    h = synth.neighbour_hamiltonian(100, 5, cutoff=4.5, seed=3)
    p, st, status = orc.trs4(h, h.meta["n_occ"], eps=1e-9, tol=1e-9)
    assert status == orc.OK
    p2, st2, s2 = orc.tc2(h, h.meta["n_occ"], eps=1e-9, tol=1e-9)
    assert _rel(p.to_dense(), p2.to_dense()) <= 1e-6
    assert st["trace_p"] == pytest.approx(h.meta["n_occ"], abs=1e-5)
    assert st["iterations"] < st2["iterations"]


# ------------------------------------------------------ submatrix method

def _exact_density(d, mu):
    w, v = np.linalg.eigh(d - mu * np.eye(d.shape[0]))
    return v[:, w < 0] @ v[:, w < 0].T


def _sym(rng, n):
    a = rng.standard_normal((n, n))
    return 0.5 * (a + a.T)


def test_submatrix_single_block_neighbourhoods_are_exact(orc):
    """Only diagonal blocks stored: every submatrix is one block, so P is the
    exact density of the block-diagonal H."""
    rng = np.random.default_rng(60)
    sizes = rng.integers(1, 8, 9)
    off = np.concatenate([[0], np.cumsum(sizes)])
    d = np.zeros((off[-1], off[-1]))
    for i in range(sizes.size):
        d[off[i]:off[i + 1], off[i]:off[i + 1]] = _sym(rng, sizes[i])
    p, rec = orc.submatrix_density(_dense_to_bsr(d, sizes), mu=0.15)
    assert rec["max_dim"] == sizes.max()
    assert _rel(p.to_dense(), _exact_density(d, 0.15)) <= 1e-12


@pytest.mark.parametrize("mu", [-0.4, 0.3])
def test_submatrix_full_pattern_is_exact(orc, mu):
    """Every block stored: every submatrix is the whole matrix, so P is the
    exact density; mu = -0.4 and 0.3 give different occupations."""
    rng = np.random.default_rng(61)
    sizes = rng.integers(1, 6, 7)
    d = _sym(rng, int(sizes.sum()))
    p, rec = orc.submatrix_density(_dense_to_bsr(d, sizes), mu=mu)
    assert rec["n_sub"] == sizes.size and rec["max_dim"] == sizes.sum()
    assert _rel(p.to_dense(), _exact_density(d, mu)) <= 1e-12


def test_submatrix_arrow_pattern(orc):
    """Block 0 coupled to every block, the others only to block 0: column 0's
    neighbourhood is everything, so P's block column 0 is exact; block
    column j != 0 comes from the two-block submatrix over {0, j}, assembled
    here by dense indexing of H."""
    rng = np.random.default_rng(62)
    sizes = rng.integers(1, 6, 6)
    off = np.concatenate([[0], np.cumsum(sizes)])
    n = int(off[-1])
    d = _sym(rng, n)
    mask = np.zeros((n, n), bool)
    for i in range(sizes.size):
        for j in range(sizes.size):
            if i == j or i == 0 or j == 0:
                mask[off[i]:off[i + 1], off[j]:off[j + 1]] = True
    d = np.where(mask, d, 0.0)
    mu = 0.05
    p, rec = orc.submatrix_density(_dense_to_bsr(d, sizes), mu=mu)
    pd = p.to_dense()
    ex = _exact_density(d, mu)
    c0 = slice(off[0], off[1])
    assert _rel(pd[:, c0], ex[:, c0]) <= 1e-12
    for j in range(1, sizes.size):
        idx = np.r_[off[0]:off[1], off[j]:off[j + 1]]
        pj = _exact_density(d[np.ix_(idx, idx)], mu)
        cj = slice(off[j], off[j + 1])
        got = pd[:, cj]
        assert np.allclose(got[idx], pj[:, sizes[0]:], atol=1e-13)
        others = np.setdiff1d(np.arange(n), idx)
        assert not got[others].any()


def test_submatrix_neighbour_hamiltonian_approximates_the_density(orc):
    """On a gapped neighbour Hamiltonian the submatrix density is close to
    the exact one (the method's approximation, not an identity): within
    1e-3 in the relative Frobenius norm, trace within 1e-3 of the occupied
    count, pattern of H; the filter then drops blocks below eps."""
    h = synth.neighbour_hamiltonian(100, 5, cutoff=4.5, seed=3)
    p, rec = orc.submatrix_density(h)
    assert np.array_equal(p.row_ptr, h.row_ptr) and np.array_equal(p.col_idx, h.col_idx)
    ex = _exact_density(h.to_dense(), 0.0)
    assert _rel(p.to_dense(), ex) <= 1e-3
    assert np.trace(p.to_dense()) == pytest.approx(h.meta["n_occ"], abs=1e-3)
    pf, _ = orc.submatrix_density(h, eps=1e-2)
    off = p.block_offsets()
    norms = {(int(i), int(j)): np.sqrt((p.values[off[t]:off[t + 1]] ** 2).sum())
             for t, (i, j) in enumerate(zip(p.block_rows(), p.col_idx))}
    kept = {(int(i), int(j)) for i, j in zip(pf.block_rows(), pf.col_idx)}
    assert kept == {k for k, v in norms.items() if v >= 1e-2} and len(kept) < len(norms)


def test_submatrix_column_sample_matches_the_full_run(orc):
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=8)
    p, _ = orc.submatrix_density(h)
    cols = [3, 17, 40]
    ps, rec = orc.submatrix_density(h, columns=cols)
    assert rec["n_sub"] == 3
    full = p.to_dense()
    part = ps.to_dense()
    off = np.concatenate([[0], np.cumsum(h.col_blk_size)])
    for j in cols:
        sl = slice(off[j], off[j + 1])
        assert np.array_equal(part[:, sl], full[:, sl])


# ------------------------------------------------ product-level norm screening

def _scale_blocks(m: BSR, rng, lo=-4.0):
    """Scale every stored block by 10^U(lo, 0) so block norms spread widely."""
    off = m.block_offsets()
    v = m.values.copy()
    for t in range(m.nnzb):
        v[off[t]:off[t + 1]] *= 10.0 ** rng.uniform(lo, 0.0)
    return BSR(m.row_blk_size, m.col_blk_size, m.row_ptr, m.col_idx, v)


def _screened_expected(alpha, a, b, beta, c, tau, eps):
    """Brute force with the screening rule: per C block of the unscreened
    pattern, the sum of the dense block products whose squared norms'
    product is not below tau^2, then alpha, beta C_in and the filter.
    Returns the kept blocks and the smallest relative distance of a norm
    product from tau^2 (ties)."""
    ab, bb = _blocks(a), _blocks(b)
    cb = _blocks(c) if (c is not None and beta != 0.0) else {}
    sa = {key: float((x * x).sum()) for key, x in ab.items()}
    sb = {key: float((x * x).sum()) for key, x in bb.items()}
    rows_of_k = {}
    for (k, j) in bb:
        rows_of_k.setdefault(k, []).append(j)
    pattern = set(cb)
    for (i, k) in ab:
        for j in rows_of_k.get(k, ()):
            pattern.add((i, j))
    t2, margin, kept = tau * tau, np.inf, {}
    for (i, j) in pattern:
        m_, n_ = int(a.row_blk_size[i]), int(b.col_blk_size[j])
        acc = np.zeros((m_, n_))
        for (ii, k), x in ab.items():
            if ii != i or (k, j) not in bb:
                continue
            p = sa[(i, k)] * sb[(k, j)]
            margin = min(margin, abs(p - t2) / t2)
            if p >= t2:
                acc += x @ bb[(k, j)]
        blk = alpha * acc + (beta * cb[(i, j)] if (i, j) in cb else 0.0)
        if not (float((blk * blk).sum()) < eps * eps):
            kept[(i, j)] = blk
    return kept, margin


@pytest.mark.parametrize("seed", range(6))
def test_multiply_screened_matches_bruteforce(orc, seed):
    rng = np.random.default_rng(300 + seed)
    nb = int(rng.integers(3, 7))
    sizes = rng.choice([3, 5, 8], nb) if seed % 2 else np.full(nb, 5)
    a = _scale_blocks(synth.random_bsr(nb, nb, sizes, sizes, 0.6, rng), rng)
    b = _scale_blocks(synth.random_bsr(nb, nb, sizes, sizes, 0.6, rng), rng)
    c = synth.random_bsr(nb, nb, sizes, sizes, 0.3, rng)
    beta = float(rng.choice([0.0, 1.5]))
    # tau at the median of the norm products, nudged off ties
    ab, bb = _blocks(a), _blocks(b)
    prods = sorted(float((x * x).sum()) * float((y * y).sum())
                   for (i, k), x in ab.items() for (kk, j), y in bb.items() if kk == k)
    tau = float(np.sqrt(prods[len(prods) // 2])) * 1.0001
    kept, margin = _screened_expected(-0.7, a, b, beta, c, tau, 0.0)
    assert margin > 1e-9
    got = orc.multiply(-0.7, a, b, beta, c, screen=tau)
    assert got.pattern() == set(kept)
    gb = _blocks(got)
    for key, blk in kept.items():
        assert _rel(gb[key], blk) <= 1e-13, key
    # screening really removed terms, and tau = 0 is the plain product
    full = orc.multiply(-0.7, a, b, beta, c)
    assert _rel(full.values, got.values) > 1e-12
    assert np.array_equal(orc.multiply(-0.7, a, b, beta, c, screen=0.0).values, full.values)


def test_sign_screened_converges_near_the_plain_sign(orc):
    """The screened Newton-Schulz iteration: with a screening threshold
    below the filter the result stays within the filter's accuracy of the
    unscreened one, and trace(P) at the occupied count."""
    h = synth.neighbour_hamiltonian(100, 5, cutoff=4.5, seed=3)
    x0, st0, s0 = orc.sign_ns(h, eps=1e-7, tol=1e-7)
    x1, st1, s1 = orc.sign_ns(h, eps=1e-7, tol=1e-7, screen=1e-9)
    assert s0 == s1 == orc.OK
    assert _rel(x1.to_dense(), x0.to_dense()) < 1e-5
    assert st1["trace_p"] == pytest.approx(h.meta["n_occ"], abs=1e-4)
    with pytest.raises(RuntimeError):
        orc.sign_ns(h, eps=1e-7, tol=1e-7, order=3, screen=1e-9)
