"""Helpers for the GPU parity tests: move synth.BSR matrices through the
C ABI and compare results with the oracle."""
import numpy as np
import pytest

from synth import BSR

# Tolerances.  FP64 results must stay within 1e-10 relative Frobenius error
# of the oracle; a single multiply reorders sums only inside one C block, so
# it is held to 1e-12.  The mixed-precision forms are held to 1e-6.
TOL_FP64_MULTIPLY = 1e-12
TOL_FP64 = 1e-10
TOL_MIXED = 1e-6


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(m: BSR):
    from paper_2003_03868_amd import bsm
    return bsm.Matrix.from_bsr(m, device=True)


def from_dev(h) -> BSR:
    rp, ci, va = h.export()
    return BSR(h.row_blk_size, h.col_blk_size, rp, ci, va)


def rel_fro(x: np.ndarray, y: np.ndarray) -> float:
    ny = float(np.linalg.norm(y))
    return float(np.linalg.norm(x - y)) / (ny if ny > 0 else 1.0)


def assert_same_matrix(got: BSR, ref: BSR, tol: float, what: str = ""):
    got.check()
    assert got.nbrows == ref.nbrows and got.nbcols == ref.nbcols
    assert np.array_equal(got.row_ptr, ref.row_ptr), f"{what}: row_ptr differs"
    assert np.array_equal(got.col_idx, ref.col_idx), f"{what}: col_idx differs"
    err = rel_fro(got.values, ref.values)
    assert err <= tol, f"{what}: relative Frobenius error {err:.3e} > {tol:.1e}"
    return err


def block_norm_margin(m: BSR, eps: float, norm: str):
    """Relative distance of every block's filter quantity from the threshold."""
    off = m.block_offsets()
    out = []
    for t in range(m.nnzb):
        x = m.values[off[t]:off[t + 1]]
        if norm == "frob":
            v, thr = float((x * x).sum()), eps * eps
        else:
            v, thr = float(np.abs(x).max()), eps
        out.append(abs(v - thr) / thr if thr > 0 else np.inf)
    return np.array(out)
