"""GPU parity of bsm_multiply / bsm_filter and the reductions against the
CPU oracle, through the C ABI."""
import os

import numpy as np
import pytest

import synth
from synth import BSR
from tests.gpu_util import (TOL_FP64_MULTIPLY, assert_same_matrix, block_norm_margin,
                            from_dev, need_gpu, rel_fro, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _case(seed, nbr, nbk, nbc, maxb, dens):
    rng = np.random.default_rng(seed)
    rs = rng.integers(1, maxb + 1, nbr)
    ks = rng.integers(1, maxb + 1, nbk)
    cs = rng.integers(1, maxb + 1, nbc)
    a = synth.random_bsr(nbr, nbk, rs, ks, dens[0], rng)
    b = synth.random_bsr(nbk, nbc, ks, cs, dens[1], rng)
    c = synth.random_bsr(nbr, nbc, rs, cs, dens[2], rng)
    return a, b, c


def _run(alpha, a, b, beta, c, eps=0.0, norm="frob"):
    from paper_2003_03868_amd import bsm
    da, db = to_dev(a), to_dev(b)
    dc = to_dev(c) if c is not None else bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    st = bsm.bsm_multiply(alpha, da.handle, db.handle, beta, dc.handle, eps,
                          bsm.NORM_FROB if norm == "frob" else bsm.NORM_MAXABS)
    out = from_dev(dc)
    for h in (da, db, dc):
        h.destroy()
    return out, st


CASES = []
_r = np.random.default_rng(99)
for _q in range(24):
    CASES.append(dict(seed=int(_r.integers(1 << 30)), nbr=int(_r.integers(1, 9)),
                      nbk=int(_r.integers(1, 9)), nbc=int(_r.integers(1, 9)),
                      maxb=int(_r.choice([1, 4, 5, 13, 16, 17, 23, 32])),
                      dens=tuple(float(x) for x in _r.choice([0.0, 0.25, 0.6, 1.0], 3)),
                      alpha=float(_r.choice([1.0, -0.5, 2.0])),
                      beta=float(_r.choice([0.0, 1.0, 1.5]))))


@pytest.mark.parametrize("case", CASES, ids=[f"r{i}" for i in range(len(CASES))])
def test_multiply_random_vs_oracle(orc, case):
    a, b, c = _case(case["seed"], case["nbr"], case["nbk"], case["nbc"], case["maxb"], case["dens"])
    ref = orc.multiply(case["alpha"], a, b, case["beta"], c)
    got, st = _run(case["alpha"], a, b, case["beta"], c)
    assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, "multiply")
    assert st.nnzb == ref.nnzb


def test_multiply_832_workload(orc):
    """64 x 64 grid of 13 x 13 blocks, 20% present, eps = 0."""
    a, b = synth.random_bsr_pair(64, 13, 0.2, seed=0)
    ref = orc.multiply(1.0, a, b)
    got, st = _run(1.0, a, b, 0.0, None)
    err = assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, "832")
    # flops and product count are integers fixed by the patterns
    pa, pb = a.pattern(), b.pattern()
    rows_of = {}
    for (k, j) in pb:
        rows_of.setdefault(k, 0)
        rows_of[k] += 1
    nprod = sum(rows_of.get(k, 0) for (_, k) in pa)
    assert st.n_products == nprod
    assert st.flops == 2.0 * 13 ** 3 * nprod
    print(f"832 multiply: err {err:.2e}, products {nprod}")


def test_multiply_chunked_matches_single(orc, monkeypatch):
    """A tiny chunk size forces many product chunks; results must not change."""
    a, b = synth.random_bsr_pair(24, 7, 0.4, seed=3)
    ref = orc.multiply(1.0, a, b)
    monkeypatch.setenv("BSM_CHUNK_PRODUCTS", "37")
    got, _ = _run(1.0, a, b, 0.0, None)
    assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, "chunked")


@pytest.mark.parametrize("norm", ["frob", "maxabs"])
@pytest.mark.parametrize("q", [0.2, 0.5, 0.9])
def test_multiply_filter_vs_oracle(orc, norm, q):
    a, b, c = _case(17, 7, 6, 7, 23, (0.6, 0.6, 0.5))
    unf = orc.multiply(1.0, a, b, 1.5, c)
    off = unf.block_offsets()
    if norm == "frob":
        vals = np.sort([np.sqrt((unf.values[off[t]:off[t + 1]] ** 2).sum()) for t in range(unf.nnzb)])
    else:
        vals = np.sort([np.abs(unf.values[off[t]:off[t + 1]]).max() for t in range(unf.nnzb)])
    eps = float(vals[int(q * (len(vals) - 1))]) * (1 + 1e-7)
    assert block_norm_margin(unf, eps, norm).min() > 1e-12   # no ties
    ref = orc.multiply(1.0, a, b, 1.5, c, eps=eps, norm=norm)
    got, st = _run(1.0, a, b, 1.5, c, eps=eps, norm=norm)
    assert st.nnzb_unfiltered == unf.nnzb
    assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, "filtered")


def test_multiply_aliasing_c_is_a(orc):
    """C may be the same handle as A (the sign update X <- 1.5X - 0.5 X Y)."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=1)
    x = orc.shift_scale(h, 0.0, 0.01)
    y = orc.multiply(1.0, x, x)
    ref = orc.multiply(-0.5, x, y, 1.5, x)
    dx, dy = to_dev(x), to_dev(y)
    bsm.bsm_multiply(-0.5, dx.handle, dy.handle, 1.5, dx.handle)
    assert_same_matrix(from_dev(dx), ref, TOL_FP64_MULTIPLY, "aliased")


def test_multiply_edge_cases(orc):
    from paper_2003_03868_amd import bsm
    a, b, c = _case(5, 4, 3, 5, 6, (0.0, 0.5, 0.5))          # empty A
    got, st = _run(1.0, a, b, 0.0, None)
    assert got.nnzb == 0 and st.n_products == 0
    got, _ = _run(1.0, a, b, 2.0, c)                         # C = 2 Cin
    assert_same_matrix(got, orc.multiply(1.0, a, b, 2.0, c), 0.0, "beta only")
    a, b, _ = _case(6, 3, 3, 3, 4, (1.0, 1.0, 0.0))
    got, _ = _run(0.0, a, b, 0.0, None)                      # alpha = 0 keeps zero blocks
    assert got.nnzb == 9 and not np.any(got.values)
    a1 = BSR(np.ones(1), np.ones(1), [0, 1], [0], [3.0])
    got, _ = _run(2.0, a1, a1, 0.0, None)                    # 1 x 1 blocks
    assert got.values.tolist() == [18.0]
    # invalid calls
    a, b, _ = _case(7, 3, 3, 3, 5, (0.5, 0.5, 0.0))
    bad = synth.random_bsr(3, 3, 9, 9, 1.0, np.random.default_rng(0))
    da, dbad = to_dev(a), to_dev(bad)
    dc = bsm.Matrix.empty_like(a.row_blk_size, bad.col_blk_size)
    with pytest.raises(bsm.BsmError) as e:
        bsm.bsm_multiply(1.0, da.handle, dbad.handle, 0.0, dc.handle)
    assert e.value.status == bsm.EINVAL
    db = to_dev(b)
    dc2 = bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    with pytest.raises(bsm.BsmError) as e:
        bsm.bsm_multiply(1.0, da.handle, db.handle, 0.0, dc2.handle, -1.0)
    assert e.value.status == bsm.EINVAL
    # non-canonical input is refused at creation
    with pytest.raises(bsm.BsmError) as e:
        bsm.Matrix.from_arrays([2, 2], [2, 2], [0, 2, 2], [1, 0], np.zeros(8))
    assert e.value.status == bsm.EINVAL
    with pytest.raises(bsm.BsmError) as e:
        bsm.Matrix.from_arrays([40], [2], [0, 1], [0], np.zeros(80))
    assert e.value.status == bsm.EINVAL


def test_multiply_nonfinite(orc):
    from paper_2003_03868_amd import bsm
    a, b, _ = _case(8, 3, 3, 3, 5, (1.0, 1.0, 0.0))
    a.values[3] = np.nan
    da, db = to_dev(a), to_dev(b)
    dc = bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    with pytest.raises(bsm.BsmError) as e:
        bsm.bsm_multiply(1.0, da.handle, db.handle, 0.0, dc.handle)
    assert e.value.status == bsm.ENONFINITE


@pytest.mark.parametrize("norm", ["frob", "maxabs"])
def test_filter_vs_oracle(orc, norm):
    from paper_2003_03868_amd import bsm
    rng = np.random.default_rng(21)
    m = synth.random_bsr(9, 9, rng.integers(1, 33, 9), rng.integers(1, 33, 9), 0.6, rng)
    m.values *= np.repeat(rng.uniform(0.0, 2.0, m.nnzb) ** 6, np.diff(m.block_offsets()))
    for eps in [0.0, 0.05, 0.5, 3.0]:
        if eps > 0:
            assert block_norm_margin(m, eps, norm).min() > 1e-12
        ref = orc.filter(m, eps, norm)
        d = to_dev(m)
        bsm.bsm_filter(d.handle, eps, bsm.NORM_FROB if norm == "frob" else bsm.NORM_MAXABS)
        assert_same_matrix(from_dev(d), ref, 0.0, f"filter {eps}")


def test_reductions_vs_oracle(orc):
    import torch
    from paper_2003_03868_amd import bsm
    rng = np.random.default_rng(22)
    sizes = rng.integers(1, 33, 12)
    m = synth.random_bsr(12, 12, sizes, sizes, 0.4, rng)
    d = to_dev(m)
    assert bsm.bsm_trace(d.handle) == pytest.approx(orc.trace(m), rel=1e-13, abs=1e-13)
    for shift in [0.0, 1.0, -2.5]:
        assert bsm.bsm_sqdist_identity(d.handle, shift) == pytest.approx(
            orc.sqdist_identity(m, shift), rel=1e-12)
        assert bsm.bsm_inf_norm(d.handle, shift) == pytest.approx(
            orc.inf_norm_shifted(m, shift), rel=1e-13)
    out = torch.zeros(m.nnzb, dtype=torch.float64, device="cuda")
    bsm.bsm_block_norms(d.handle, out)
    torch.cuda.synchronize()
    assert np.allclose(out.cpu().numpy(), orc.block_sqnorms(m), rtol=1e-13, atol=0)
    # shift/scale with a missing diagonal block inserted
    rp, ci = m.row_ptr.copy(), m.col_idx.copy()
    has_diag = [any(ci[rp[i]:rp[i + 1]] == i) for i in range(12)]
    assert not all(has_diag)
    h2 = bsm.bsm_shift_scale(d.handle, 0.7, 0.25)
    got = from_dev(bsm.Matrix(h2, sizes, sizes))
    assert_same_matrix(got, orc.shift_scale(m, 0.7, 0.25), 1e-15, "shift_scale")


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 6])
@pytest.mark.parametrize("maxb", [5, 13, 23, 26, 32])
def test_multiply_kernel_variants(orc, monkeypatch, variant, maxb):
    """All FP64 block-product kernels (16x16 tiles, 4x4 tiles, fixed shapes)
    against the oracle, uniform and mixed block sizes up to maxb."""
    monkeypatch.setenv("BSM_SMM_VARIANT", str(variant))
    for seed, uniform in [(31, True), (32, False)]:
        rng = np.random.default_rng(seed + maxb)
        nb = 9
        if uniform:
            rs = ks = cs = np.full(nb, maxb)
        else:
            rs, ks, cs = (rng.integers(1, maxb + 1, nb) for _ in range(3))
        a = synth.random_bsr(nb, nb, rs, ks, 0.5, rng)
        b = synth.random_bsr(nb, nb, ks, cs, 0.5, rng)
        c = synth.random_bsr(nb, nb, rs, cs, 0.3, rng)
        ref = orc.multiply(-0.5, a, b, 1.5, c)
        got, _ = _run(-0.5, a, b, 1.5, c)
        assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, f"variant {variant} maxb {maxb}")


@pytest.mark.parametrize("group,waves,stage", [("2", "1", "1"), ("2", "2", "1"), ("2", "4", "1"),
                                                ("2", "4", "2"), ("4", "16", "1"), ("42", "8", "1")])
@pytest.mark.parametrize("b", [5, 6, 13, 23, 26, 32])
def test_quad_kernel_vs_oracle_and_fixed(orc, monkeypatch, group, waves, stage, b):
    """The group kernel (2 x 2 quads with one, two or four waves, one or two
    entries staged per step; 4 x 4 groups with sixteen waves; 4 x 2 groups
    with eight waves for size 23; merged
    product lists) against the oracle -- block-row and column counts that
    are not multiples of the group edge give partial groups, C_in adds
    blocks without products, a tiny chunk size and an odd band height give
    many chunks, and the symbolic walk is split into three k segments -- and
    bit for bit against the one-C-block-per-wave
    compile-time-shape kernel, which sums the same products in the same
    order with the same instructions."""
    monkeypatch.setenv("BSM_QUAD_GROUP", group)
    monkeypatch.setenv("BSM_QUAD_WAVES", waves)
    monkeypatch.setenv("BSM_QUAD_STAGE", stage)
    rng = np.random.default_rng(500 + b)
    nbr, nbk, nbc = 11, 9, 13
    a = synth.random_bsr(nbr, nbk, np.full(nbr, b), np.full(nbk, b), 0.45, rng)
    bm = synth.random_bsr(nbk, nbc, np.full(nbk, b), np.full(nbc, b), 0.45, rng)
    c = synth.random_bsr(nbr, nbc, np.full(nbr, b), np.full(nbc, b), 0.3, rng)
    for alpha, beta, cc in [(1.0, 0.0, None), (-0.5, 1.5, c)]:
        ref = orc.multiply(alpha, a, bm, beta, cc)
        monkeypatch.setenv("BSM_SMM_VARIANT", "6")
        got, st = _run(alpha, a, bm, beta, cc)
        assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, f"quad b={b} beta={beta}")
        monkeypatch.setenv("BSM_SMM_VARIANT", "2")
        fixed, _ = _run(alpha, a, bm, beta, cc)
        assert np.array_equal(got.values, fixed.values), "quad and fixed kernels differ"
        monkeypatch.setenv("BSM_SMM_VARIANT", "6")
        monkeypatch.setenv("BSM_CHUNK_PRODUCTS", "50")
        monkeypatch.setenv("BSM_TILE_ROWS", "3")
        monkeypatch.setenv("BSM_QUAD_KSEG", "3")      # three k segments per row group
        chunked, st2 = _run(alpha, a, bm, beta, cc)
        assert st2.smm_launches > 1
        assert np.array_equal(chunked.values, got.values), "chunks or k segments changed the result"
        monkeypatch.delenv("BSM_CHUNK_PRODUCTS")
        monkeypatch.delenv("BSM_TILE_ROWS")
        monkeypatch.delenv("BSM_QUAD_KSEG")


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_multiply_mixed_class_sizes(orc, monkeypatch, variant):
    """Block sizes drawn from {5, 13, 23, 26}: the per-class launches (4), the
    fused persistent launch (3) and the run-time-shape kernel (1) agree with
    the oracle, also with several chunks."""
    monkeypatch.setenv("BSM_SMM_VARIANT", str(variant))
    rng = np.random.default_rng(77)
    nb = 14
    rs, ks, cs = (rng.choice([5, 13, 23, 26], nb) for _ in range(3))
    a = synth.random_bsr(nb, nb, rs, ks, 0.5, rng)
    b = synth.random_bsr(nb, nb, ks, cs, 0.5, rng)
    c = synth.random_bsr(nb, nb, rs, cs, 0.3, rng)
    ref = orc.multiply(1.0, a, b, -0.5, c)
    got, _ = _run(1.0, a, b, -0.5, c)
    assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, f"variant {variant}")
    monkeypatch.setenv("BSM_CHUNK_PRODUCTS", "300")
    monkeypatch.setenv("BSM_TILE_ROWS", "2")
    got, _ = _run(1.0, a, b, -0.5, c)
    assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, f"variant {variant} chunked")


@pytest.mark.parametrize("stage", ["1", "2"])
@pytest.mark.parametrize("shape", [(45, 29, 37), (70, 70, 70), (3, 5, 2)], ids=["rect", "square", "tiny"])
def test_mixed_quads_vs_oracle_and_class_kernel(orc, monkeypatch, shape, stage):
    """Mixed sizes from {5, 13, 23, 26} through the paired-group kernel (one
    persistent launch over every (m, n) class): the oracle's product, and
    bit for bit the per-class kernels' (the default for such sizes), which
    sum the same products in the same order with the same instructions.
    Row and column counts that leave rows unpaired, C_in blocks without
    products, many chunks (bands of 32 rows) and three k segments; one or
    two entries staged per barrier pair (an odd entry count leaves the
    second stage empty)."""
    monkeypatch.setenv("BSM_MQUAD_STAGE", stage)
    nbr, nbk, nbc = shape
    rng = np.random.default_rng(900 + nbr)
    rs, ks, cs = (rng.choice([5, 13, 23, 26], n) for n in (nbr, nbk, nbc))
    a = synth.random_bsr(nbr, nbk, rs, ks, 0.4, rng)
    b = synth.random_bsr(nbk, nbc, ks, cs, 0.4, rng)
    c = synth.random_bsr(nbr, nbc, rs, cs, 0.3, rng)
    for alpha, beta, cc in [(1.0, 0.0, None), (-0.5, 1.5, c)]:
        ref = orc.multiply(alpha, a, b, beta, cc)
        monkeypatch.setenv("BSM_SMM_VARIANT", "7")
        got, st = _run(alpha, a, b, beta, cc)
        assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, f"mixed quads {shape} beta={beta}")
        for v in ("4", "6"):
            monkeypatch.setenv("BSM_SMM_VARIANT", v)
            cls, _ = _run(alpha, a, b, beta, cc)
            assert np.array_equal(got.values, cls.values), "mixed quads and class kernels differ"
        monkeypatch.setenv("BSM_SMM_VARIANT", "7")
        monkeypatch.setenv("BSM_CHUNK_PRODUCTS", "200")
        monkeypatch.setenv("BSM_QUAD_KSEG", "3")
        chunked, st2 = _run(alpha, a, b, beta, cc)
        if nbr > 32:
            assert st2.smm_launches > 1
        assert np.array_equal(chunked.values, got.values), "chunks or k segments changed the result"
        monkeypatch.delenv("BSM_CHUNK_PRODUCTS")
        monkeypatch.delenv("BSM_QUAD_KSEG")


CATALOGUE = [(f, w, p) for f in (0, 1) for w in (1, 2, 4) for p in (0, 1)]


@pytest.mark.parametrize("entry", CATALOGUE, ids=lambda e: f"f{e[0]}w{e[1]}p{e[2]}")
def test_tuned_kernel_parameters_vs_oracle(orc, monkeypatch, entry):
    """Every tunable kernel parameter set gives the oracle's product, for a
    uniform size without a fixed-shape kernel and for mixed class sizes."""
    from paper_2003_03868_amd import bsm
    monkeypatch.setenv("BSM_SMM_VARIANT", "5")
    rng = np.random.default_rng(303)
    nb = 11
    for rs, ks, cs in [(np.full(nb, 17), np.full(nb, 9), np.full(nb, 30)),
                       tuple(rng.integers(1, 33, nb) for _ in range(3))]:
        a = synth.random_bsr(nb, nb, rs, ks, 0.5, rng)
        b = synth.random_bsr(nb, nb, ks, cs, 0.5, rng)
        c = synth.random_bsr(nb, nb, rs, cs, 0.3, rng)
        key = (int(rs.max()), int(cs.max()), int(ks.max()) if (rs == rs[0]).all() else 0)
        bsm.bsm_set_smm_table([((int(rs[0]), int(cs[0]), int(ks[0])), entry), (key, entry)])
        try:
            ref = orc.multiply(1.5, a, b, -1.0, c)
            got, _ = _run(1.5, a, b, -1.0, c)
        finally:
            bsm.bsm_set_smm_table(None)
        assert_same_matrix(got, ref, TOL_FP64_MULTIPLY, f"entry {entry}")
    # class launches with a run-time kernel chosen by the table
    monkeypatch.setenv("BSM_SMM_VARIANT", "4")
    rs, ks, cs = (rng.choice([5, 13, 23, 26], nb) for _ in range(3))
    a = synth.random_bsr(nb, nb, rs, ks, 0.5, rng)
    b = synth.random_bsr(nb, nb, ks, cs, 0.5, rng)
    bsm.bsm_set_smm_table([((m, n, 0), entry) for m in (5, 13, 23, 26) for n in (5, 13, 23, 26)])
    try:
        got, _ = _run(1.0, a, b, 0.0, None)
    finally:
        bsm.bsm_set_smm_table(None)
    assert_same_matrix(got, orc.multiply(1.0, a, b), TOL_FP64_MULTIPLY, f"class {entry}")


def test_smm_bench_entry_point():
    from paper_2003_03868_amd import bsm
    cat = CATALOGUE + [(2, 1, 1)]
    ms = bsm.bsm_smm_bench(23, 13, 26, 500, 16, cat, reps=2)
    assert len(ms) == len(cat) and all(t > 0 for t in ms)
    ms = bsm.bsm_smm_bench(23, 13, 0, 300, 8, cat, reps=1)   # mixed k
    assert all(t > 0 for t in ms)
    with pytest.raises(bsm.BsmError):
        bsm.bsm_smm_bench(40, 5, 5, 10, 4, CATALOGUE, reps=1)
    with pytest.raises(bsm.BsmError):
        bsm.bsm_smm_bench(7, 5, 5, 10, 4, [(2, 1, 1)], reps=1)   # no class kernel for 7
    with pytest.raises(bsm.BsmError):
        bsm.bsm_set_smm_table([((5, 5, 5), (4, 1, 1))])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_transpose_vs_oracle(orc, seed):
    """A^T on the GPU against the oracle, bit for bit (data movement only):
    rectangular, mixed block sizes up to 32, empty rows and columns; twice
    gives A back."""
    from paper_2003_03868_amd import bsm
    rng = np.random.default_rng(900 + seed)
    nbr, nbc = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    a = synth.random_bsr(nbr, nbc, rng.integers(1, 33, nbr), rng.integers(1, 33, nbc),
                         [0.0, 0.05, 0.3, 0.9][seed], rng)
    ref = orc.transpose(a)
    da = to_dev(a)
    th = bsm.bsm_transpose(da.handle)
    t = bsm.Matrix(th, a.col_blk_size, a.row_blk_size)
    got = from_dev(t)
    for f in ("row_ptr", "col_idx", "values"):
        assert np.array_equal(getattr(got, f), getattr(ref, f)), f
    bh = bsm.bsm_transpose(t.handle)
    back = from_dev(bsm.Matrix(bh, a.row_blk_size, a.col_blk_size))
    for f in ("row_ptr", "col_idx", "values"):
        assert np.array_equal(getattr(back, f), getattr(a, f)), f


def test_transpose_of_the_full_sign_hamiltonian_is_itself(orc):
    """H of the sign workload is symmetric: H^T == H bit for bit at full size
    (2048 sites x 23, 187,560 blocks)."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(2048, 23, density=0.1, cutoff=6.0, seed=0)
    dh = to_dev(h)
    t = from_dev(bsm.Matrix(bsm.bsm_transpose(dh.handle), h.col_blk_size, h.row_blk_size))
    for f in ("row_ptr", "col_idx", "values"):
        assert np.array_equal(getattr(t, f), getattr(h, f)), f
