"""CPU oracle (plain C, FP64) for the block-sparse multiply and sign iteration.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the HIP library or its binding.
The C source (``bsm_oracle.c``) is compiled with gcc into ``liboracle.so``
next to it; it shares no code with the HIP path.  Matrices travel as
``synth.BSR`` objects (plain arrays from the input generator).

Parity status of each function (what pins it, see ``tests/test_oracle.py``):

* ``multiply``      -- pinned: dense NumPy GEMM brute force on random tiny
                       cases (mixed sizes, alpha/beta, filter), the block
                       pattern by Python set logic; with screening, the same
                       brute force leaving out the screened terms.
* ``filter``        -- pinned: keep rule re-derived per block from the dense
                       matrix.
* ``sign_ns``       -- pinned: eigen-decomposition sign (LAPACK) on tiny
                       dense cases, scalar recurrence on diagonal H, 2x2
                       closed form, trace = number of negative eigenvalues.
* ``trace``, ``sqdist_identity``, ``inf_norm_shifted`` -- pinned against
                       ``numpy`` on the dense matrix.
* ``add``           -- pinned: dense NumPy sum, pattern union, keep rule.
* ``transpose``     -- pinned: the dense transpose (NumPy) on rectangular
                       mixed-size cases with empty rows and columns; twice
                       is the identity, bit for bit.
* ``sign_ns`` orders 3, 5, 7 -- pinned: the printed polynomials (order 7:
                       derived in the test from its closed form) on diagonal
                       H, eigen-decomposition sign on tiny dense cases.
* ``sqrt_inv``      -- pinned: eigen-decomposition S^{+-1/2} (LAPACK) on tiny
                       dense SPD cases; the scalar coupled recurrence on
                       diagonal S by hand.
* ``density_nonorth`` -- pinned: P from the generalised eigenproblem
                       K c = e S c (LAPACK) on tiny cases; P S P = P and
                       trace(P S) = occupied count on filtered neighbour cases.
* ``tc2``           -- pinned: diagonal H by hand (the scalar maps and the
                       trace decisions); on dense cases the projector onto
                       the N lowest eigenvectors (LAPACK).
* ``trs4``          -- pinned: on diagonal H one update maps every entry by
                       one member of the fourth-order family with the trace
                       reset to N (gamma recovered from one entry, checked on
                       the rest), the branch rules by hand; on dense cases the
                       projector onto the N lowest eigenvectors (LAPACK), and
                       TC2's result.
* ``submatrix_density`` -- pinned: exact (the full eigendecomposition
                       density) when every column's neighbourhood is the
                       whole matrix or a single block, and on the hub column
                       of an arrow pattern; brute-force dense assembly of
                       each submatrix on tiny cases.
* ``mu_bisect``     -- pinned: diagonal H, whose count is the number of
                       diagonal entries below mu, so every midpoint follows
                       by hand; on dense cases the accepted mu lies in the
                       eigenvalue gap that gives the target count (LAPACK).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

from synth import BSR

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsm_oracle.c")
# A test may point this at a deliberately broken copy to show the pins fail.
_LIB = os.environ.get("BSM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

NORM_FROB, NORM_MAXABS = 0, 1
OK, EINVAL, ENOMEM, ENOCONV, ENONFINITE = 0, -1, -2, -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _OMat(C.Structure):
    _fields_ = [("nbrows", C.c_int32), ("nbcols", C.c_int32),
                ("rbs", C.c_void_p), ("cbs", C.c_void_p),
                ("nnzb", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("values", C.c_void_p)]


class _SignStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_multiplies", C.c_int32),
                ("r_hist", C.c_double * 128), ("scale", C.c_double),
                ("trace_x", C.c_double), ("trace_p", C.c_double),
                ("flops", C.c_double), ("nnzb_x", C.c_int64 * 128),
                ("nnzb_y", C.c_int64 * 128)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            lib = C.CDLL(_LIB)
            P = C.POINTER(_OMat)
            lib.orc_multiply.argtypes = [C.c_double, P, P, C.c_double, P, C.c_double, C.c_int, P]
            lib.orc_filter.argtypes = [P, C.c_double, C.c_int, P]
            lib.orc_block_sqnorms.argtypes = [P, C.c_void_p]
            lib.orc_trace.argtypes = [P]
            lib.orc_trace.restype = C.c_double
            lib.orc_sqdist_identity.argtypes = [P, C.c_double]
            lib.orc_sqdist_identity.restype = C.c_double
            lib.orc_inf_norm_shifted.argtypes = [P, C.c_double]
            lib.orc_inf_norm_shifted.restype = C.c_double
            lib.orc_shift_scale.argtypes = [P, C.c_double, C.c_double, P]
            lib.orc_sign_ns.argtypes = [P, C.c_double, C.c_double, C.c_int, C.c_double,
                                        C.c_int32, C.c_int32, P, C.POINTER(_SignStats)]
            lib.orc_sign.argtypes = [P, C.c_double, C.c_double, C.c_int, C.c_double,
                                     C.c_int32, C.c_int32, C.c_int32, C.c_double, P,
                                     C.POINTER(_SignStats)]
            lib.orc_multiply_screened.argtypes = [C.c_double, P, P, C.c_double, P, C.c_double,
                                                  C.c_int, C.c_double, P]
            lib.orc_add.argtypes = [C.c_double, P, C.c_double, P, C.c_double, C.c_double,
                                    C.c_int, P]
            lib.orc_transpose.argtypes = [P, P]
            lib.orc_density_from_sign.argtypes = [P, P]
            lib.orc_tc2.argtypes = [P, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int32,
                                    P, C.POINTER(_Tc2Stats)]
            lib.orc_trs4.argtypes = [P, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int32,
                                     P, C.POINTER(_Tc2Stats)]
            lib.orc_sqrt_inv.argtypes = [P, C.c_double, C.c_int, C.c_double, C.c_int32, P, P,
                                         C.POINTER(_SignStats)]
            lib.orc_density_nonorth.argtypes = [P, P, C.c_double, C.c_double, C.c_int,
                                                C.c_double, C.c_int32, C.c_int32, P,
                                                C.POINTER(C.c_double), C.POINTER(_SignStats),
                                                C.POINTER(_SignStats)]
            lib.orc_free.argtypes = [P]
            lib.orc_num_threads.restype = C.c_int
            lib.orc_set_threads.argtypes = [C.c_int]
            _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def _in(m: BSR) -> tuple[_OMat, tuple]:
    keep = (m.row_blk_size, m.col_blk_size, m.row_ptr, m.col_idx, m.values)
    om = _OMat(m.nbrows, m.nbcols, _ptr(m.row_blk_size), _ptr(m.col_blk_size),
               m.nnzb, _ptr(m.row_ptr), _ptr(m.col_idx), _ptr(m.values))
    return om, keep


def _out(om: _OMat, rbs: np.ndarray, cbs: np.ndarray) -> BSR:
    lib = _load()
    nnzb = int(om.nnzb)
    rp = np.ctypeslib.as_array(C.cast(om.row_ptr, C.POINTER(C.c_int64)), (om.nbrows + 1,)).copy()
    ci = (np.ctypeslib.as_array(C.cast(om.col_idx, C.POINTER(C.c_int32)), (nnzb,)).copy()
          if nnzb else np.zeros(0, np.int32))
    rows = np.repeat(np.arange(om.nbrows), np.diff(rp))
    nval = int((rbs[rows].astype(np.int64) * cbs[ci].astype(np.int64)).sum())
    vals = (np.ctypeslib.as_array(C.cast(om.values, C.POINTER(C.c_double)), (nval,)).copy()
            if nval else np.zeros(0))
    lib.orc_free(C.byref(om))
    return BSR(rbs.copy(), cbs.copy(), rp, ci, vals)


def _check(st: int, what: str):
    if st != OK:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def _norm(norm) -> int:
    return {"frob": NORM_FROB, "maxabs": NORM_MAXABS, NORM_FROB: NORM_FROB,
            NORM_MAXABS: NORM_MAXABS}[norm]


def multiply(alpha: float, a: BSR, b: BSR, beta: float = 0.0, c: BSR | None = None,
             eps: float = 0.0, norm="frob", screen: float = 0.0) -> BSR:
    """C = alpha*A*B + beta*Cin, then the block-norm filter (plain loops);
    screen > 0 leaves out the terms with ||A_ik||^2 ||B_kj||^2 < screen^2."""
    lib = _load()
    oa, ka = _in(a)
    ob, kb = _in(b)
    oc, kc = _in(c) if c is not None else (None, None)
    out = _OMat()
    cref = C.byref(oc) if oc is not None else None
    if screen > 0.0:
        st = lib.orc_multiply_screened(alpha, C.byref(oa), C.byref(ob), beta, cref, eps,
                                       _norm(norm), screen, C.byref(out))
    else:
        st = lib.orc_multiply(alpha, C.byref(oa), C.byref(ob), beta, cref, eps, _norm(norm),
                              C.byref(out))
    _check(st, "multiply")
    return _out(out, a.row_blk_size, b.col_blk_size)


def filter(a: BSR, eps: float, norm="frob") -> BSR:  # noqa: A001 - mirrors the operation name
    lib = _load()
    oa, ka = _in(a)
    out = _OMat()
    _check(lib.orc_filter(C.byref(oa), eps, _norm(norm), C.byref(out)), "filter")
    return _out(out, a.row_blk_size, a.col_blk_size)


def block_sqnorms(a: BSR) -> np.ndarray:
    lib = _load()
    oa, ka = _in(a)
    out = np.zeros(a.nnzb)
    _check(lib.orc_block_sqnorms(C.byref(oa), _ptr(out)), "block_sqnorms")
    return out


def trace(a: BSR) -> float:
    oa, ka = _in(a)
    return float(_load().orc_trace(C.byref(oa)))


def sqdist_identity(a: BSR, shift: float = 1.0) -> float:
    oa, ka = _in(a)
    return float(_load().orc_sqdist_identity(C.byref(oa), shift))


def inf_norm_shifted(a: BSR, mu: float = 0.0) -> float:
    oa, ka = _in(a)
    return float(_load().orc_inf_norm_shifted(C.byref(oa), mu))


def shift_scale(a: BSR, mu: float, scale: float) -> BSR:
    lib = _load()
    oa, ka = _in(a)
    out = _OMat()
    _check(lib.orc_shift_scale(C.byref(oa), mu, scale, C.byref(out)), "shift_scale")
    return _out(out, a.row_blk_size, a.col_blk_size)


def add(alpha: float, a: BSR, beta: float = 0.0, b: BSR | None = None, gamma: float = 0.0,
        eps: float = 0.0, norm="frob") -> BSR:
    """C = alpha A + beta B + gamma I (pattern union), then the filter."""
    lib = _load()
    oa, ka = _in(a)
    ob, kb = _in(b) if b is not None else (None, None)
    out = _OMat()
    _check(lib.orc_add(alpha, C.byref(oa), beta, C.byref(ob) if ob is not None else None,
                       gamma, eps, _norm(norm), C.byref(out)), "add")
    return _out(out, a.row_blk_size, a.col_blk_size)


def transpose(a: BSR) -> BSR:
    """A^T: block (i, j) becomes block (j, i), transposed."""
    lib = _load()
    oa, ka = _in(a)
    out = _OMat()
    _check(lib.orc_transpose(C.byref(oa), C.byref(out)), "transpose")
    return _out(out, a.col_blk_size, a.row_blk_size)


def sign_ns(h: BSR, mu: float = 0.0, eps: float = 0.0, tol: float = 1e-6,
            max_iter: int = 100, fixed_iters: int = 0, norm="frob", order: int = 2,
            screen: float = 0.0):
    """Sign iteration of the given order (2: Newton-Schulz, 3, 5, 7); returns
    (X, stats, status).

    ``status`` is OK, ENOCONV or ENONFINITE; X is the last iterate in every
    case that produced one.
    """
    lib = _load()
    oh, kh = _in(h)
    out = _OMat()
    st = _SignStats()
    status = lib.orc_sign(C.byref(oh), mu, eps, _norm(norm), tol, max_iter, fixed_iters, order,
                          screen, C.byref(out), C.byref(st))
    if status not in (OK, ENOCONV, ENONFINITE):
        raise RuntimeError(f"oracle sign iteration failed with status {status}")
    x = _out(out, h.row_blk_size, h.col_blk_size) if out.row_ptr else None
    stats = dict(iterations=int(st.iterations), n_multiplies=int(st.n_multiplies),
                 r_hist=[float(st.r_hist[k]) for k in range(st.iterations + 1)],
                 scale=float(st.scale), trace_x=float(st.trace_x),
                 trace_p=float(st.trace_p), flops=float(st.flops),
                 nnzb_x=[int(st.nnzb_x[k]) for k in range(st.iterations + 1)],
                 nnzb_y=[int(st.nnzb_y[k]) for k in range(st.iterations + 1)])
    return x, stats, int(status)


def _submatrix_module():
    """oracle/submatrix.py, or the copy BSM_ORACLE_SUBMATRIX names (a test
    points it at a deliberately broken copy to show the pins fail)."""
    path = os.environ.get("BSM_ORACLE_SUBMATRIX")
    if not path:
        from . import submatrix
        return submatrix
    import importlib.util
    spec = importlib.util.spec_from_file_location("oracle_submatrix_variant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def submatrix_density(h: BSR, mu: float = 0.0, eps: float = 0.0, norm="frob", columns=None):
    """P by the submatrix method (see oracle/submatrix.py); returns (P, record)."""
    return _submatrix_module().submatrix_density(h, mu=mu, eps=eps, norm=norm, columns=columns)


def mu_bisect(h: BSR, n_target: float, mu_lo: float, mu_hi: float, count_tol: float = 0.5,
              max_steps: int = 40, **sign_kw):
    """Chemical potential for a fixed electron count by bisection on
    trace(P(mu)) = (n - trace sign(H - mu I))/2 (the extra iterations the
    Density-matrix-based-methods paragraph says a canonical ensemble needs):
    mu = (lo + hi)/2; count from the sign iteration at mu; stop when
    |count - n_target| <= count_tol, else lo = mu (count < n_target) or
    hi = mu.  The endpoints are never evaluated.  Returns (mu, X, record,
    status) with status OK or ENOCONV (no midpoint within count_tol)."""
    lo, hi = float(mu_lo), float(mu_hi)
    rec = dict(mu_hist=[], count_hist=[], sign_noconv=0)
    x = None
    for _ in range(max_steps):
        mu = 0.5 * (lo + hi)
        x, st, status = sign_ns(h, mu=mu, **sign_kw)
        if status not in (OK, ENOCONV):
            raise RuntimeError(f"oracle sign iteration failed with status {status}")
        rec["sign_noconv"] += status == ENOCONV
        count = st["trace_p"]
        rec["mu_hist"].append(mu)
        rec["count_hist"].append(count)
        if abs(count - n_target) <= count_tol:
            return mu, x, rec, OK
        if count < n_target:
            lo = mu
        else:
            hi = mu
    return mu, x, rec, ENOCONV


class _Tc2Stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_multiplies", C.c_int32),
                ("e_hist", C.c_double * 128), ("branch", C.c_int32 * 128),
                ("scale", C.c_double), ("trace_p", C.c_double), ("flops", C.c_double),
                ("gamma_hist", C.c_double * 128)]


def _purify(fn, h: BSR, n_occ: float, eps: float, tol: float, max_iter: int, norm):
    lib = _load()
    oh, kh = _in(h)
    out = _OMat()
    st = _Tc2Stats()
    status = getattr(lib, fn)(C.byref(oh), float(n_occ), eps, _norm(norm), tol, max_iter,
                              C.byref(out), C.byref(st))
    if status not in (OK, ENOCONV, ENONFINITE):
        raise RuntimeError(f"oracle purification failed with status {status}")
    p = _out(out, h.row_blk_size, h.col_blk_size) if out.row_ptr else None
    k = int(st.iterations)
    stats = dict(iterations=k, n_multiplies=int(st.n_multiplies),
                 e_hist=[float(st.e_hist[i]) for i in range(k + 1)],
                 branch=[int(st.branch[i]) for i in range(k)],
                 gamma=[float(st.gamma_hist[i]) for i in range(k)], scale=float(st.scale),
                 trace_p=float(st.trace_p), flops=float(st.flops))
    return p, stats, int(status)


def tc2(h: BSR, n_occ: float, eps: float = 0.0, tol: float = 1e-10, max_iter: int = 100,
        norm="frob"):
    """Trace-correcting purification (orc_tc2); returns (P, stats, status)
    with status OK, ENOCONV or ENONFINITE."""
    return _purify("orc_tc2", h, n_occ, eps, tol, max_iter, norm)


def trs4(h: BSR, n_occ: float, eps: float = 0.0, tol: float = 1e-10, max_iter: int = 100,
         norm="frob"):
    """Trace-resetting fourth-order purification (orc_trs4); returns
    (P, stats, status) as tc2, with stats["gamma"] the gamma of each update
    and branch 2 for the fourth-order map."""
    return _purify("orc_trs4", h, n_occ, eps, tol, max_iter, norm)


def _stats(st) -> dict:
    return dict(iterations=int(st.iterations), n_multiplies=int(st.n_multiplies),
                r_hist=[float(st.r_hist[k]) for k in range(st.iterations + 1)],
                scale=float(st.scale), trace_x=float(st.trace_x),
                trace_p=float(st.trace_p), flops=float(st.flops))


def sqrt_inv(s: BSR, eps: float = 0.0, tol: float = 1e-10, max_iter: int = 100, norm="frob"):
    """S^{1/2} and S^{-1/2} of a symmetric positive definite S by the coupled
    Newton-Schulz iteration (orc_sqrt_inv); returns (sqrt, inv_sqrt, stats,
    status) with status OK or ENOCONV."""
    lib = _load()
    oh, kh = _in(s)
    o1, o2 = _OMat(), _OMat()
    st = _SignStats()
    status = lib.orc_sqrt_inv(C.byref(oh), eps, _norm(norm), tol, max_iter, C.byref(o1),
                              C.byref(o2), C.byref(st))
    if status not in (OK, ENOCONV):
        raise RuntimeError(f"oracle square-root iteration failed with status {status}")
    return (_out(o1, s.row_blk_size, s.col_blk_size), _out(o2, s.row_blk_size, s.col_blk_size),
            _stats(st), int(status))


def density_nonorth(k: BSR, s: BSR, mu: float = 0.0, eps: float = 0.0, tol: float = 1e-10,
                    max_iter: int = 100, norm="frob", order: int = 2):
    """P = (I - sign(S^{-1} K - mu I)) S^{-1} / 2 through the symmetric form
    Z (I - sign(Z K Z - mu I)) Z / 2 with Z = S^{-1/2} (orc_density_nonorth);
    returns (P, trace(P S), sqrt stats, sign stats, status)."""
    lib = _load()
    ok_, kk = _in(k)
    os_, ks = _in(s)
    out = _OMat()
    tps = C.c_double()
    s1, s2 = _SignStats(), _SignStats()
    status = lib.orc_density_nonorth(C.byref(ok_), C.byref(os_), mu, eps, _norm(norm), tol,
                                     max_iter, order, C.byref(out), C.byref(tps), C.byref(s1),
                                     C.byref(s2))
    if status not in (OK, ENOCONV):
        raise RuntimeError(f"oracle non-orthogonal density failed with status {status}")
    return (_out(out, k.row_blk_size, k.col_blk_size), float(tps.value), _stats(s1), _stats(s2),
            int(status))


def density_from_sign(x: BSR) -> BSR:
    lib = _load()
    ox, kx = _in(x)
    out = _OMat()
    _check(lib.orc_density_from_sign(C.byref(ox), C.byref(out)), "density_from_sign")
    return _out(out, x.row_blk_size, x.col_blk_size)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of later oracle calls (for timing; results do not change)."""
    _load().orc_set_threads(int(n))
