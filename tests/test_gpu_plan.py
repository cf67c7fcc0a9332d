"""Planned multiplies: bsm_multiply_plan keeps the symbolic results of a
multiply, bsm_plan_execute repeats only its numeric kernels (no allocation,
copy or wait) for new operand values with the same patterns.

A repeat runs the kernels of the normal multiply on the same symbolic data,
so its result must equal, bit for bit, bsm_multiply of the same values (and
the oracle to the single-multiply tolerance); a repeat captured into a
hipGraph must do the same on every replay, with eager work in between.  The
record of the executes flags a filter that would keep another block set."""
import numpy as np
import pytest

import synth
from tests.gpu_util import TOL_FP64_MULTIPLY, assert_same_matrix, from_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _revalue(m: synth.BSR, seed: int, scale: float = 1.0) -> synth.BSR:
    """The same pattern with new N(0,1) values (times scale)."""
    rng = np.random.default_rng(seed)
    return synth.BSR(m.row_blk_size, m.col_blk_size, m.row_ptr, m.col_idx,
                     scale * rng.standard_normal(m.values.shape[0]))


def _multiply(a, b, eps, prec=0):
    from paper_2003_03868_amd import bsm
    da, db = to_dev(a), to_dev(b)
    dc = bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    bsm.bsm_multiply(1.0, da.handle, db.handle, 0.0, dc.handle, eps, bsm.NORM_FROB, prec)
    return from_dev(dc)


CASES = [
    dict(name="quad13", nb=40, size=13, eps=0.0, prec=0),
    dict(name="quad23_filtered", nb=24, size=23, eps=1e-9, prec=0),
    dict(name="mixed", nb=40, size=(5, 13, 23, 26), eps=0.0, prec=0),
    dict(name="fp32", nb=32, size=13, eps=0.0, prec=1),
    dict(name="bf16x3", nb=32, size=23, eps=0.0, prec=3),
]


def _pair(c, seed):
    if isinstance(c["size"], tuple):
        rng = np.random.default_rng(seed)
        sizes = rng.choice(np.array(c["size"], dtype=np.int32), size=c["nb"])
        a = synth.random_bsr(c["nb"], c["nb"], sizes, sizes, 0.25, rng)
        b = synth.random_bsr(c["nb"], c["nb"], sizes, sizes, 0.25, rng)
        return a, b
    return synth.random_bsr_pair(c["nb"], c["size"], 0.25, seed=seed)


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_plan_repeats_equal_multiply(orc, c):
    from paper_2003_03868_amd import bsm
    a, b = _pair(c, seed=5)
    da, db = to_dev(a), to_dev(b)
    dc = bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    plan, st = bsm.bsm_multiply_plan(1.0, da.handle, db.handle, dc.handle, c["eps"],
                                     prec=c["prec"])
    try:
        first = from_dev(dc)
        assert_same_matrix(first, _multiply(a, b, c["eps"], c["prec"]), 0.0, "planning call")
        for r in range(3):
            a2, b2 = _revalue(a, 100 + r), _revalue(b, 200 + r)
            da2, db2 = to_dev(a2), to_dev(b2)
            bsm.bsm_plan_execute(plan, da2.handle, db2.handle, dc.handle)
            assert bsm.bsm_plan_status(plan) == 0
            got = from_dev(dc)
            ref = _multiply(a2, b2, c["eps"], c["prec"])
            assert np.array_equal(got.row_ptr, first.row_ptr)
            assert np.array_equal(got.values, ref.values), f"repeat {r} differs from bsm_multiply"
            if c["prec"] == 0:
                assert_same_matrix(got, orc.multiply(1.0, a2, b2, eps=c["eps"]),
                                   TOL_FP64_MULTIPLY, "plan repeat vs oracle")
            da2.destroy()
            db2.destroy()
    finally:
        bsm.bsm_plan_destroy(plan)


def test_plan_square_and_checks():
    """A = B (the square of the sign iteration), then the checks of execute:
    C with another pattern, distinct operands for a square's plan, C = A."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 13, cutoff=4.0, seed=2)
    dh = to_dev(h)
    dc = bsm.Matrix.empty_like(h.row_blk_size, h.col_blk_size)
    plan, _ = bsm.bsm_multiply_plan(1.0, dh.handle, dh.handle, dc.handle, 0.0)
    try:
        h2 = _revalue(h, 7)
        dh2 = to_dev(h2)
        bsm.bsm_plan_execute(plan, dh2.handle, dh2.handle, dc.handle)
        assert np.array_equal(from_dev(dc).values, _multiply(h2, h2, 0.0).values)
        other = bsm.Matrix.empty_like(h.row_blk_size, h.col_blk_size)
        with pytest.raises(bsm.BsmError) as e:
            bsm.bsm_plan_execute(plan, dh2.handle, dh2.handle, other.handle)
        assert e.value.status == bsm.EINVAL
        with pytest.raises(bsm.BsmError) as e:
            bsm.bsm_plan_execute(plan, dh2.handle, dh.handle, dc.handle)
        assert e.value.status == bsm.EINVAL
        with pytest.raises(bsm.BsmError) as e:
            bsm.bsm_plan_execute(plan, dh2.handle, dh2.handle, dh2.handle)
        assert e.value.status == bsm.EINVAL
    finally:
        bsm.bsm_plan_destroy(plan)
    with pytest.raises(bsm.BsmError):
        bsm.bsm_multiply_plan(1.0, dh.handle, dh.handle, dh.handle, 0.0)


def test_plan_flags_a_changed_keep_set():
    """Doubling the operands quadruples every block's squared norm: with the
    threshold at the median product block, blocks just below it would now be
    kept, which the record reports; the same values again report nothing."""
    from paper_2003_03868_amd import bsm
    a, b = synth.random_bsr_pair(32, 13, 0.25, seed=9)
    full = _multiply(a, b, 0.0)
    off = full.block_offsets()
    norms = np.array([np.linalg.norm(full.values[off[t]:off[t + 1]]) for t in range(full.nnzb)])
    eps = float(np.median(norms))
    assert np.any((norms < eps) & (norms >= eps / 2))
    da, db = to_dev(a), to_dev(b)
    dc = bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    plan, _ = bsm.bsm_multiply_plan(1.0, da.handle, db.handle, dc.handle, eps)
    try:
        bsm.bsm_plan_execute(plan, da.handle, db.handle, dc.handle)
        assert bsm.bsm_plan_status(plan) == 0
        a2 = synth.BSR(a.row_blk_size, a.col_blk_size, a.row_ptr, a.col_idx, 2.0 * a.values)
        da2 = to_dev(a2)
        bsm.bsm_plan_execute(plan, da2.handle, db.handle, dc.handle)
        assert bsm.bsm_plan_status(plan) == 2
        assert bsm.bsm_plan_status(plan) == 0      # the report cleared the record
    finally:
        bsm.bsm_plan_destroy(plan)


def test_plan_execute_in_a_captured_graph():
    """One execute captured into a hipGraph (through torch's stream capture),
    replayed three times; before each replay an eager execute with other
    operands overwrites C, so every replay must recompute A B."""
    import torch
    from paper_2003_03868_amd import bsm
    a, b = synth.random_bsr_pair(48, 13, 0.25, seed=11)
    a2, b2 = _revalue(a, 1), _revalue(b, 2)
    da, db, da2, db2 = to_dev(a), to_dev(b), to_dev(a2), to_dev(b2)
    dc = bsm.Matrix.empty_like(a.row_blk_size, b.col_blk_size)
    plan, _ = bsm.bsm_multiply_plan(1.0, da.handle, db.handle, dc.handle, 0.0)
    try:
        ref = from_dev(dc).values.copy()
        ref2 = _multiply(a2, b2, 0.0).values
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                bsm.bsm_plan_execute(plan, da.handle, db.handle, dc.handle,
                                     stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        for r in range(3):
            bsm.bsm_plan_execute(plan, da2.handle, db2.handle, dc.handle)
            torch.cuda.synchronize()
            assert np.array_equal(from_dev(dc).values, ref2), f"eager execute before replay {r}"
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(from_dev(dc).values, ref), f"replay {r}"
        assert bsm.bsm_plan_status(plan) == 0
        del g
    finally:
        bsm.bsm_plan_destroy(plan)
