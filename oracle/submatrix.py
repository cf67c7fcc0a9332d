"""Submatrix method (section "Submatrix Method"; CPU oracle, test
infrastructure only).

The density matrix is assembled one block column at a time from small dense
problems: for block column j, the principal submatrix of H over the block
rows stored in column j (block j itself and its neighbours) is formed
densely, its own density matrix is taken through a full eigendecomposition
(the form the paper's comparison with the Newton-Schulz iteration uses),
and that matrix's block column of j becomes block column j of P, on H's
pattern.  Plain loops over block columns; ``numpy.linalg.eigh`` is the only
library step.

Readings (none of them fixed by the text):
* the index set of column j is the block rows with a stored block in
  column j, in ascending order;
* P_j = (I - sign(T_j - mu I)) / 2 with T_j the dense submatrix; an
  eigenvalue exactly at mu gets sign 0;
* P has H's block pattern and is filtered with the block-norm rule after
  assembly.
"""
from __future__ import annotations

import numpy as np

from synth import BSR


def column_sets(h: BSR) -> list[np.ndarray]:
    """Block rows i with a stored block H_ij, per block column j (ascending)."""
    rows = h.block_rows()
    sets = [[] for _ in range(h.nbcols)]
    for t in range(h.nnzb):
        sets[int(h.col_idx[t])].append(int(rows[t]))
    return [np.array(sorted(s), dtype=np.int64) for s in sets]


def _blocks(h: BSR) -> dict:
    off = h.block_offsets()
    rows = h.block_rows()
    out = {}
    for t in range(h.nnzb):
        i, j = int(rows[t]), int(h.col_idx[t])
        out[(i, j)] = h.values[off[t]:off[t + 1]].reshape(h.row_blk_size[i], h.col_blk_size[j])
    return out


def submatrix_dense(h: BSR, idx: np.ndarray, blocks: dict | None = None) -> np.ndarray:
    """The dense principal submatrix of H over the block indices idx."""
    blocks = _blocks(h) if blocks is None else blocks
    sz = h.row_blk_size[idx].astype(np.int64)
    st = np.concatenate([[0], np.cumsum(sz)])
    t = np.zeros((st[-1], st[-1]))
    for a, i in enumerate(idx):
        for b, j in enumerate(idx):
            blk = blocks.get((int(i), int(j)))
            if blk is not None:
                t[st[a]:st[a + 1], st[b]:st[b + 1]] = blk
    return t


def submatrix_density(h: BSR, mu: float = 0.0, eps: float = 0.0, norm: str = "frob",
                      columns=None):
    """P by the submatrix method; returns (P, record).

    ``columns`` (optional) restricts the work to those block columns: P then
    holds only their blocks (a sample for timing or spot checks)."""
    if h.nbrows != h.nbcols or not np.array_equal(h.row_blk_size, h.col_blk_size):
        raise ValueError("H must be square with square diagonal blocks")
    blocks = _blocks(h)
    sets = column_sets(h)
    cols = range(h.nbcols) if columns is None else [int(c) for c in columns]
    out = {}
    dims = []
    for j in cols:
        idx = sets[j]
        t = submatrix_dense(h, idx, blocks)
        t -= mu * np.eye(t.shape[0])
        w, v = np.linalg.eigh(t)
        x = (v * np.sign(w)) @ v.T
        pj = 0.5 * (np.eye(t.shape[0]) - x)
        sz = h.row_blk_size[idx].astype(np.int64)
        st = np.concatenate([[0], np.cumsum(sz)])
        a = int(np.searchsorted(idx, j))
        assert idx[a] == j, "a stored diagonal block is required"
        for b, i in enumerate(idx):
            out[(int(i), j)] = pj[st[b]:st[b + 1], st[a]:st[a + 1]]
        dims.append(t.shape[0])
    # assemble on H's pattern (restricted to the requested columns), then filter
    keep_rp, keep_ci, vals = [0], [], []
    for i in range(h.nbrows):
        cnt = 0
        for t in range(int(h.row_ptr[i]), int(h.row_ptr[i + 1])):
            j = int(h.col_idx[t])
            blk = out.get((i, j))
            if blk is None:
                continue
            if eps > 0.0:
                drop = ((blk * blk).sum() < eps * eps) if norm == "frob" else (np.abs(blk).max() < eps)
                if drop:
                    continue
            keep_ci.append(j)
            vals.append(blk.ravel())
            cnt += 1
        keep_rp.append(keep_rp[-1] + cnt)
    p = BSR(h.row_blk_size.copy(), h.col_blk_size.copy(), np.array(keep_rp, dtype=np.int64),
            np.array(keep_ci, dtype=np.int32),
            np.concatenate(vals) if vals else np.zeros(0))
    rec = dict(n_sub=len(dims), dims=dims, max_dim=max(dims) if dims else 0,
               flops_eigh=float(sum(9.0 * d ** 3 for d in dims)))
    return p, rec
