"""The residual reduction that allocates nothing (bsm_sqdist_identity_noalloc)
against bsm_sqdist_identity, through the C ABI: the same kernels in the same
order, so the same bits; two calls in a row, the second on a smaller matrix
(the fixed scratch keeps the first call's partial sums, which the second must
not see); an empty matrix; and the capacity error beyond 2^20 block rows."""
import numpy as np
import pytest

import synth
from tests.gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _noalloc(bsm, torch, h, shift):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    st = bsm.bsm_sqdist_identity_noalloc(h.handle, shift, out.data_ptr(), stream=stream)
    torch.cuda.synchronize()
    return st, float(out.item())


def test_noalloc_residual_matches_allocating_entry_point():
    import torch
    from paper_2003_03868_amd import bsm
    big = synth.neighbour_hamiltonian(300, 23, cutoff=5.0, seed=4)
    small = synth.neighbour_hamiltonian(120, 13, cutoff=4.0, seed=5)
    for m, shift in ((big, 1.0), (small, 0.5)):
        d = to_dev(m)
        st, got = _noalloc(bsm, torch, d, shift)
        assert st == bsm.OK, bsm.bsm_last_error()
        ref = bsm.bsm_sqdist_identity(d.handle, shift)
        assert got == ref, (got, ref)
        dense = m.to_dense() - shift * np.eye(m.shape[0])
        assert abs(got - float((dense * dense).sum())) <= 1e-12 * got
        d.destroy()
    # a block-diagonal-free matrix: the shift of every missing diagonal block
    sz = np.full(7, 5, np.int32)
    e = synth.BSR(sz, sz, np.zeros(8, np.int64), np.zeros(0, np.int32), np.zeros(0))
    de = to_dev(e)
    st, got = _noalloc(bsm, torch, de, 2.0)
    assert st == bsm.OK and got == bsm.bsm_sqdist_identity(de.handle, 2.0) == 35 * 4.0


def test_noalloc_residual_capacity_and_empty():
    import torch
    from paper_2003_03868_amd import bsm
    n = (1 << 20) + 1
    sz = np.ones(n, np.int32)
    big = synth.BSR(sz, sz, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    d = to_dev(big)
    st, got = _noalloc(bsm, torch, d, 1.0)
    assert st == bsm.ECAPACITY and np.isnan(got)
    assert "scratch" in bsm.bsm_last_error()
    d.destroy()
    z = np.zeros(0, np.int32)
    empty = synth.BSR(z, z, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    de = to_dev(empty)
    st, got = _noalloc(bsm, torch, de, 1.0)
    assert st == bsm.OK and got == 0.0
