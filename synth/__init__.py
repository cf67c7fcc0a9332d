"""Seeded synthetic inputs for the block-sparse multiply and the sign iteration.

This package only *makes inputs*: random block-sparse matrices in blocked-CSR
(BSR) form.  It holds none of the method's arithmetic (no products, no
filtering, no sign iteration) and imports neither the CPU oracle nor the HIP
library, so both sides can be fed the very same arrays.

BSR layout used throughout (the blocked CSR format of the DBCSR section):

* ``row_blk_size[nbrows]``, ``col_blk_size[nbcols]`` -- int32 block sizes;
* ``row_ptr[nbrows + 1]`` -- int64, block-row pointers into ``col_idx``;
* ``col_idx[nnzb]`` -- int32, strictly increasing inside each block row;
* ``values`` -- float64, the stored blocks concatenated in CSR order, each
  block ``row_blk_size[i] x col_blk_size[j]`` in row-major order.

Recipes (all seeded through ``numpy.random.default_rng(seed)``):

* :func:`random_bsr` -- every block position independently present with
  probability ``density``, entries N(0, 1).  The 832 x 832 single-multiply
  workload is ``random_bsr_pair(64, 13, 0.2, seed)``.
* :func:`neighbour_hamiltonian` -- sites uniformly at random in a periodic
  cube at a given number density, one block per site whose size comes from the
  atomic basis, blocks present when the minimum-image distance is below the
  cutoff, entries ``exp(-0.5 r) * N(0, 1)``, symmetrised, and the diagonal
  shifted by +-Delta so that a gap is certified around mu = 0 (Gershgorin).
* :func:`overlap_like` -- a symmetric positive definite overlap matrix S with
  the block pattern of a symmetric matrix: I plus decaying random couplings
  scaled so that Gershgorin keeps the spectrum in [1 - tau, 1 + tau].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "BSR", "random_bsr", "random_bsr_pair", "neighbour_hamiltonian", "overlap_like",
    "n_occ_for_block", "config_workload", "mnk_stack", "probe_vectors",
]


@dataclass
class BSR:
    """A block-sparse matrix in canonical blocked-CSR form (host arrays)."""

    row_blk_size: np.ndarray
    col_blk_size: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.row_blk_size = np.ascontiguousarray(self.row_blk_size, dtype=np.int32)
        self.col_blk_size = np.ascontiguousarray(self.col_blk_size, dtype=np.int32)
        self.row_ptr = np.ascontiguousarray(self.row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(self.col_idx, dtype=np.int32)
        self.values = np.ascontiguousarray(self.values, dtype=np.float64)

    @property
    def nbrows(self) -> int:
        return int(self.row_blk_size.shape[0])

    @property
    def nbcols(self) -> int:
        return int(self.col_blk_size.shape[0])

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def shape(self) -> tuple[int, int]:
        return int(self.row_blk_size.sum()), int(self.col_blk_size.sum())

    def block_rows(self) -> np.ndarray:
        """Block-row index of every stored block (int64)."""
        return np.repeat(np.arange(self.nbrows, dtype=np.int64), np.diff(self.row_ptr))

    def block_offsets(self) -> np.ndarray:
        """Offset of every stored block inside ``values`` (length nnzb + 1)."""
        sz = self.row_blk_size[self.block_rows()].astype(np.int64) * \
            self.col_blk_size[self.col_idx].astype(np.int64)
        off = np.zeros(self.nnzb + 1, dtype=np.int64)
        np.cumsum(sz, out=off[1:])
        return off

    def check(self) -> None:
        """Raise ValueError unless the arrays form a canonical BSR matrix."""
        if self.row_ptr.shape[0] != self.nbrows + 1 or self.row_ptr[0] != 0:
            raise ValueError("row_ptr must have nbrows+1 entries starting at 0")
        if np.any(np.diff(self.row_ptr) < 0) or self.row_ptr[-1] != self.nnzb:
            raise ValueError("row_ptr must be non-decreasing and end at nnzb")
        if self.nnzb:
            if self.col_idx.min() < 0 or self.col_idx.max() >= self.nbcols:
                raise ValueError("col_idx out of range")
            r = self.block_rows()
            same = r[1:] == r[:-1]
            if np.any(self.col_idx[1:][same] <= self.col_idx[:-1][same]):
                raise ValueError("col_idx must be strictly increasing per row")
        if self.values.shape[0] != self.block_offsets()[-1]:
            raise ValueError("values length does not match the block sizes")

    def to_dense(self) -> np.ndarray:
        """Dense float64 copy (for tiny matrices in tests)."""
        ro = np.concatenate([[0], np.cumsum(self.row_blk_size, dtype=np.int64)])
        co = np.concatenate([[0], np.cumsum(self.col_blk_size, dtype=np.int64)])
        d = np.zeros((ro[-1], co[-1]))
        off = self.block_offsets()
        rows = self.block_rows()
        for t in range(self.nnzb):
            i, j = rows[t], self.col_idx[t]
            m, n = self.row_blk_size[i], self.col_blk_size[j]
            d[ro[i]:ro[i] + m, co[j]:co[j] + n] = \
                self.values[off[t]:off[t + 1]].reshape(m, n)
        return d

    def pattern(self) -> set[tuple[int, int]]:
        return set(zip(self.block_rows().tolist(), self.col_idx.tolist()))

    def copy(self) -> "BSR":
        return BSR(self.row_blk_size.copy(), self.col_blk_size.copy(),
                   self.row_ptr.copy(), self.col_idx.copy(),
                   self.values.copy(), dict(self.meta))


def _from_pattern(row_sizes, col_sizes, present: np.ndarray, rng) -> BSR:
    """Build a BSR from a boolean block mask, entries N(0,1) in CSR order."""
    nbr, nbc = present.shape
    rows, cols = np.nonzero(present)            # row-major order == CSR order
    row_ptr = np.zeros(nbr + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nbr), out=row_ptr[1:])
    sizes = row_sizes[rows].astype(np.int64) * col_sizes[cols].astype(np.int64)
    values = rng.standard_normal(int(sizes.sum()))
    return BSR(row_sizes, col_sizes, row_ptr, cols.astype(np.int32), values)


def random_bsr(nbrows: int, nbcols: int, row_sizes, col_sizes,
               density: float, rng) -> BSR:
    """Each block position present independently with probability density."""
    row_sizes = np.broadcast_to(np.asarray(row_sizes, dtype=np.int32), (nbrows,)).copy()
    col_sizes = np.broadcast_to(np.asarray(col_sizes, dtype=np.int32), (nbcols,)).copy()
    present = rng.random((nbrows, nbcols)) < density
    return _from_pattern(row_sizes, col_sizes, present, rng)


def random_bsr_pair(nblk: int = 64, bsize: int = 13, density: float = 0.2,
                    seed: int = 0) -> tuple[BSR, BSR]:
    """Two independent square block-sparse matrices from one generator, A first.

    With the defaults this is the 832 x 832 single-multiply workload: a 64 x 64
    grid of 13 x 13 blocks, about 20% of block positions present, N(0,1)
    entries.
    """
    rng = np.random.default_rng(seed)
    a = random_bsr(nblk, nblk, bsize, bsize, density, rng)
    b = random_bsr(nblk, nblk, bsize, bsize, density, rng)
    return a, b


def n_occ_for_block(b: int) -> int:
    """Occupied orbitals per site: about 4 of every 23, at least one.

    Gives 1, 2, 4, 5 for block sizes 5, 13, 23, 26, i.e. 17-20% occupied,
    inside the 10-20% occupied-orbital range the paper quotes.
    """
    return max(1, int(np.floor(4.0 * b / 23.0 + 0.5)))


def _morton_order(pos: np.ndarray, box: float, bits: int = 10) -> np.ndarray:
    q = np.minimum((pos / box * (1 << bits)).astype(np.int64), (1 << bits) - 1)
    code = np.zeros(pos.shape[0], dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return np.argsort(code, kind="stable")


def _neighbour_pairs(pos: np.ndarray, box: float, cutoff: float):
    """All pairs I<J with minimum-image distance < cutoff (strict), sorted."""
    n = pos.shape[0]
    ii, jj, rr = [], [], []
    chunk = max(1, 2_000_000 // max(n, 1))
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d = pos[s:e, None, :] - pos[None, :, :]
        d -= box * np.round(d / box)
        r = np.sqrt((d * d).sum(-1))
        i_loc, j = np.nonzero(r < cutoff)
        i = i_loc + s
        keep = j > i
        ii.append(i[keep]); jj.append(j[keep]); rr.append(r[i_loc[keep], j[keep]])
    ii = np.concatenate(ii); jj = np.concatenate(jj); rr = np.concatenate(rr)
    order = np.lexsort((jj, ii))
    return ii[order], jj[order], rr[order]


def neighbour_hamiltonian(n_sites: int, block_sizes=23, density: float = 0.1,
                          cutoff: float = 6.0, seed: int = 0,
                          size_choices=None, gap_factor: float = 1.05,
                          spatial_sort: bool = True) -> BSR:
    """Synthetic symmetric neighbour-list Hamiltonian with a certified gap.

    Draw order from ``default_rng(seed)``: block sizes (only when
    ``size_choices`` is given, uniformly from it), site positions, then the
    diagonal blocks in site order, then the pair blocks I<J in lexicographic
    order.  Sites are renumbered along a Morton curve before the blocks are
    drawn (``spatial_sort``) so that neighbouring sites get nearby indices.

    ``H_II = (G + G^T)/2``, ``H_IJ = exp(-0.5 r_IJ) G_IJ`` for r < cutoff,
    ``H_JI = H_IJ^T``.  Then, with ``M = max`` scalar-row abs-sum of that H and
    ``Delta = gap_factor * M``, the first ``n_occ(b)`` orbitals of every site
    get ``-Delta`` on the diagonal and the rest ``+Delta``.  Every Gershgorin
    disc then excludes 0, so the number of negative eigenvalues is exactly
    ``sum n_occ`` -- the expected trace of P = (I - sign(H))/2.
    """
    rng = np.random.default_rng(seed)
    if size_choices is not None:
        sizes = rng.choice(np.asarray(size_choices, dtype=np.int32), n_sites)
    else:
        sizes = np.full(n_sites, int(block_sizes), dtype=np.int32)
    box = (n_sites / density) ** (1.0 / 3.0)
    if cutoff >= box / 2:
        raise ValueError("cutoff must be below half the box for a unique minimum image")
    pos = rng.uniform(0.0, box, (n_sites, 3))
    if spatial_sort:
        order = _morton_order(pos, box)
        pos = pos[order]
        sizes = sizes[order]
    sizes = sizes.astype(np.int32)
    pi, pj, pr = _neighbour_pairs(pos, box, cutoff)

    # Block list: diagonal + both triangles, CSR order.
    diag = np.arange(n_sites, dtype=np.int64)
    rows = np.concatenate([diag, pi, pj])
    cols = np.concatenate([diag, pj, pi])
    kind = np.concatenate([np.zeros(n_sites, np.int8), np.ones(pi.size, np.int8),
                           np.full(pi.size, 2, np.int8)])
    src = np.concatenate([diag, np.arange(pi.size), np.arange(pi.size)])
    order = np.lexsort((cols, rows))
    rows, cols, kind, src = rows[order], cols[order], kind[order], src[order]
    bsz = sizes[rows].astype(np.int64) * sizes[cols].astype(np.int64)
    off = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(bsz, out=off[1:])
    values = np.empty(int(off[-1]))
    pos_of = np.empty((3, max(n_sites, pi.size)), dtype=np.int64)
    pos_of[kind, src] = np.arange(rows.size)

    # Diagonal blocks in site order.
    for s in range(n_sites):
        b = int(sizes[s])
        g = rng.standard_normal((b, b))
        t = pos_of[0, s]
        values[off[t]:off[t + 1]] = ((g + g.T) * 0.5).ravel()
    # Pair blocks in lexicographic (I, J) order.
    scale = np.exp(-0.5 * pr)
    uniform = size_choices is None
    if uniform and pi.size:
        b = int(sizes[0])
        g_all = rng.standard_normal((pi.size, b, b)) * scale[:, None, None]
        up = pos_of[1, :pi.size]
        lo = pos_of[2, :pi.size]
        vv = values[:off[-1]].reshape(-1)
        idx = off[up][:, None] + np.arange(b * b)[None, :]
        vv[idx] = g_all.reshape(pi.size, -1)
        idx = off[lo][:, None] + np.arange(b * b)[None, :]
        vv[idx] = np.transpose(g_all, (0, 2, 1)).reshape(pi.size, -1)
    else:
        for p in range(pi.size):
            bi, bj = int(sizes[pi[p]]), int(sizes[pj[p]])
            g = rng.standard_normal((bi, bj)) * scale[p]
            t = pos_of[1, p]
            values[off[t]:off[t + 1]] = g.ravel()
            t = pos_of[2, p]
            values[off[t]:off[t + 1]] = g.T.ravel()

    row_ptr = np.zeros(n_sites + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_sites), out=row_ptr[1:])
    h = BSR(sizes, sizes, row_ptr, cols.astype(np.int32), values)

    # Scalar row abs-sums -> Delta; shift the diagonal.
    scal_off = np.concatenate([[0], np.cumsum(sizes, dtype=np.int64)])
    rowsum = np.zeros(int(scal_off[-1]))
    for t in range(rows.size):
        i, j = rows[t], cols[t]
        m, n = int(sizes[i]), int(sizes[j])
        blk = values[off[t]:off[t + 1]].reshape(m, n)
        rowsum[scal_off[i]:scal_off[i] + m] += np.abs(blk).sum(1)
    delta = gap_factor * float(rowsum.max())
    nocc_total = 0
    for s in range(n_sites):
        b = int(sizes[s])
        t = pos_of[0, s]
        blk = values[off[t]:off[t + 1]].reshape(b, b)
        no = n_occ_for_block(b)
        nocc_total += no
        d = np.full(b, delta)
        d[:no] = -delta
        blk[np.arange(b), np.arange(b)] += d
    h.meta.update(dict(n_sites=n_sites, box=box, cutoff=cutoff, density=density,
                       delta=delta, n_occ=nocc_total, seed=seed,
                       positions=pos, n_pairs=int(pi.size)))
    return h


def config_workload(name: str, seed: int = 0, scale: float = 1.0):
    """Named workloads; ``scale`` < 1 shrinks the site count for tests.

    * ``"mult832"``  -- (A, B) random 64x64 grid of 13x13 blocks, 20% present.
    * ``"sign23"``   -- 2048-site, 23x23-block neighbour Hamiltonian,
      cutoff 6 A, density 0.1 / A^3.
    * ``"mixed"``    -- 4096 sites with block sizes drawn from {5,13,23,26}.
    """
    if name == "mult832":
        return random_bsr_pair(64, 13, 0.2, seed)
    if name == "sign23":
        return neighbour_hamiltonian(max(8, int(round(2048 * scale))), 23, seed=seed)
    if name == "mixed":
        return neighbour_hamiltonian(max(8, int(round(4096 * scale))), seed=seed,
                                     size_choices=(5, 13, 23, 26))
    raise KeyError(name)


def mnk_stack(m: int, n: int, k: int, n_products: int, n_c_blocks: int,
              seed: int = 0):
    """A synthetic product stack for one (m, n, k): random A, B blocks and a
    C-block id per product (sorted by C block, the C-stationary order)."""
    rng = np.random.default_rng(seed)
    n_a = max(1, n_products // 4)
    n_b = max(1, n_products // 4)
    a = rng.standard_normal(n_a * m * k)
    b = rng.standard_normal(n_b * k * n)
    c_of = np.sort(rng.integers(0, n_c_blocks, n_products)).astype(np.int32)
    ai = rng.integers(0, n_a, n_products).astype(np.int32)
    bi = rng.integers(0, n_b, n_products).astype(np.int32)
    return a, b, ai, bi, c_of


def probe_vectors(n: int, count: int = 2, seed: int = 0) -> np.ndarray:
    """``count`` seeded Gaussian vectors of length ``n`` (rows of the result),
    for sketching a large matrix X by the products X v."""
    return np.random.default_rng(seed).standard_normal((count, n))


def overlap_like(h: BSR, tau: float = 0.5, seed: int = 0) -> BSR:
    """Overlap matrix S = I + tau * N / M with the block pattern of ``h``.

    ``h`` must have a symmetric block pattern with square diagonal blocks.
    N is symmetric: for each stored pair I < J a block ``G_IJ * w_IJ`` with
    ``G_IJ ~ N(0, 1)`` (drawn in CSR order of the upper triangle) and
    ``N_JI = N_IJ^T``; diagonal blocks ``(G_II + G_II^T)/2`` with a zero
    diagonal.  ``w_IJ = exp(-r_IJ)`` with the minimum-image site distance
    when ``h.meta`` holds positions and a box, else 1.  M is the largest
    scalar row abs-sum of N, so every Gershgorin disc of S lies in
    [1 - tau, 1 + tau] and S is positive definite for tau < 1.
    """
    if not 0.0 <= tau < 1.0:
        raise ValueError("tau must be in [0, 1)")
    rng = np.random.default_rng(seed)
    rows = h.block_rows()
    cols = h.col_idx.astype(np.int64)
    off = h.block_offsets()
    rbs, cbs = h.row_blk_size, h.col_blk_size
    if h.nbrows != h.nbcols or not np.array_equal(rbs, cbs) or \
            int((rows == cols).sum()) != h.nbrows:
        raise ValueError("h must be square with every diagonal block stored")
    pos, box = h.meta.get("positions"), h.meta.get("box")
    where = {(int(i), int(j)): t for t, (i, j) in enumerate(zip(rows, cols))}
    values = np.zeros_like(h.values)
    for t in range(h.nnzb):
        i, j = int(rows[t]), int(cols[t])
        if i > j:
            continue
        m, n = int(rbs[i]), int(cbs[j])
        w = 1.0
        if pos is not None and box is not None and i != j:
            d = pos[i] - pos[j]
            d -= box * np.round(d / box)
            w = float(np.exp(-np.sqrt(float(d @ d))))
        g = rng.standard_normal((m, n)) * w
        if i == j:
            g = 0.5 * (g + g.T)
            g[np.arange(m), np.arange(m)] = 0.0
        values[off[t]:off[t + 1]] = g.ravel()
        if i != j:
            tt = where.get((j, i))
            if tt is None:
                raise ValueError("the block pattern of h must be symmetric")
            values[off[tt]:off[tt + 1]] = g.T.ravel()
    # scalar row abs-sums of N
    scal = np.concatenate([[0], np.cumsum(rbs, dtype=np.int64)])
    rowsum = np.zeros(int(scal[-1]))
    for t in range(h.nnzb):
        i, j = int(rows[t]), int(cols[t])
        m, n = int(rbs[i]), int(cbs[j])
        rowsum[scal[i]:scal[i] + m] += np.abs(values[off[t]:off[t + 1]].reshape(m, n)).sum(1)
    big = float(rowsum.max()) if rowsum.size else 0.0
    if big > 0.0:
        values *= tau / big
    for t in range(h.nnzb):
        i, j = int(rows[t]), int(cols[t])
        if i == j:
            m = int(rbs[i])
            blk = values[off[t]:off[t + 1]].reshape(m, m)
            blk[np.arange(m), np.arange(m)] += 1.0
    s = BSR(rbs.copy(), cbs.copy(), h.row_ptr.copy(), h.col_idx.copy(), values)
    s.meta.update(dict(tau=tau, seed=seed))
    return s
