"""Python binding of libbsm: the C entry points under the same names
(argument marshalling only -- every step runs in the HIP library) plus a
small ``Matrix`` handle wrapper.

PyTorch supplies device memory for inputs/outputs and the HIP stream.  There
is no fallback: if ``libbsm.so`` is missing or cannot be loaded, importing the
library raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsm.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ENONFINITE, ECAPACITY = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, SPLIT_BF16, SPLIT_BF16X3 = 0, 1, 2, 3
NORM_FROB, NORM_MAXABS = 0, 1
STATUS_NAMES = {0: "BSM_OK", -1: "BSM_EINVAL", -2: "BSM_ENOMEM", -3: "BSM_EDEVICE",
                -4: "BSM_ENOCONV", -5: "BSM_ENONFINITE", -6: "BSM_ECAPACITY"}


class BsmError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class bsm_info(C.Structure):
    _fields_ = [("nbrows", C.c_int32), ("nbcols", C.c_int32), ("nnzb", C.c_int64),
                ("nvalues", C.c_int64), ("nrows", C.c_int64), ("ncols", C.c_int64)]


class bsm_mult_stats(C.Structure):
    _fields_ = [("n_products", C.c_int64), ("flops", C.c_double),
                ("nnzb_unfiltered", C.c_int64), ("nnzb", C.c_int64),
                ("smm_ms", C.c_double), ("total_ms", C.c_double),
                ("smm_launches", C.c_int32), ("pad_", C.c_int32), ("n_screened", C.c_int64),
                ("class_ms", C.c_double * 16)]


class bsm_sign_opts(C.Structure):
    _fields_ = [("eps_filter", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("fixed_iters", C.c_int32), ("norm", C.c_int32), ("prec", C.c_int32),
                ("fp64_final_iters", C.c_int32), ("use_graph", C.c_int32),
                ("prec_switch_tol", C.c_double), ("order", C.c_int32), ("pad_", C.c_int32),
                ("eps_screen", C.c_double)]


class bsm_sign_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_multiplies", C.c_int32),
                ("r_hist", C.c_double * 128), ("prec_hist", C.c_int32 * 128),
                ("scale", C.c_double), ("trace_x", C.c_double), ("trace_p", C.c_double),
                ("flops", C.c_double), ("n_products", C.c_int64), ("smm_ms", C.c_double),
                ("device_ms", C.c_double), ("nnzb_final", C.c_int64),
                ("graph_replays", C.c_int32), ("graph_fallbacks", C.c_int32),
                ("smm_launches", C.c_int32), ("pad_", C.c_int32),
                ("n_screened", C.c_int64), ("nnzb_x_hist", C.c_int64 * 128),
                ("nnzb_y_hist", C.c_int64 * 128), ("class_ms", C.c_double * 16)]


class bsm_mu_stats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("sign_noconv", C.c_int32),
                ("mu_hist", C.c_double * 64), ("count_hist", C.c_double * 64),
                ("flops", C.c_double), ("device_ms", C.c_double)]


class bsm_tc2_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_multiplies", C.c_int32),
                ("e_hist", C.c_double * 128), ("branch", C.c_int32 * 128),
                ("scale", C.c_double), ("trace_p", C.c_double), ("flops", C.c_double),
                ("n_products", C.c_int64), ("smm_ms", C.c_double), ("device_ms", C.c_double),
                ("gamma_hist", C.c_double * 128)]


class bsm_sub_stats(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("max_dim", C.c_int32), ("mean_dim", C.c_double),
                ("max_iterations", C.c_int32), ("n_batches", C.c_int32), ("flops", C.c_double),
                ("gemm_ms", C.c_double), ("device_ms", C.c_double), ("r_max", C.c_double),
                ("nnzb", C.c_int64)]


class bsm_smm_params(C.Structure):
    _fields_ = [("family", C.c_int32), ("wpg", C.c_int32), ("prefetch", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None
_lock = threading.Lock()

# (name, restype, argtypes) of every exported entry point
_SIGS = [
    ("bsm_sign_opts_default", None, [C.POINTER(bsm_sign_opts)]),
    ("bsm_create", C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    ("bsm_destroy", C.c_int, [C.c_void_p]),
    ("bsm_get_info", C.c_int, [C.c_void_p, C.POINTER(bsm_info)]),
    ("bsm_export", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    ("bsm_multiply", C.c_int, [C.c_double, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                               C.c_double, C.c_int32, C.c_int32, C.POINTER(bsm_mult_stats),
                               C.c_void_p]),
    ("bsm_multiply_screened", C.c_int, [C.c_double, C.c_void_p, C.c_void_p, C.c_double,
                                        C.c_void_p, C.c_double, C.c_int32, C.c_double,
                                        C.POINTER(bsm_mult_stats), C.c_void_p]),
    ("bsm_multiply_plan", C.c_int, [C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_int32, C.c_int32, C.POINTER(C.c_void_p),
                                    C.POINTER(bsm_mult_stats), C.c_void_p]),
    ("bsm_plan_execute", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("bsm_plan_status", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    ("bsm_plan_destroy", C.c_int, [C.c_void_p]),
    ("bsm_filter", C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_void_p]),
    ("bsm_block_norms", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("bsm_trace", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    ("bsm_sqdist_identity", C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    ("bsm_sqdist_identity_noalloc", C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    ("bsm_shift_scale", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_void_p),
                                  C.c_void_p]),
    ("bsm_inf_norm", C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    ("bsm_sign_iterate", C.c_int, [C.c_void_p, C.c_double, C.POINTER(bsm_sign_opts),
                                   C.POINTER(C.c_void_p), C.POINTER(bsm_sign_stats), C.c_void_p]),
    ("bsm_add", C.c_int, [C.c_double, C.c_void_p, C.c_double, C.c_void_p, C.c_double,
                          C.c_double, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p]),
    ("bsm_mu_bisect", C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                C.c_int32, C.POINTER(bsm_sign_opts), C.POINTER(C.c_double),
                                C.POINTER(C.c_void_p), C.POINTER(bsm_mu_stats), C.c_void_p]),
    ("bsm_sqrt_inv", C.c_int, [C.c_void_p, C.POINTER(bsm_sign_opts), C.POINTER(C.c_void_p),
                               C.POINTER(C.c_void_p), C.POINTER(bsm_sign_stats), C.c_void_p]),
    ("bsm_density_nonorth", C.c_int, [C.c_void_p, C.c_void_p, C.c_double,
                                      C.POINTER(bsm_sign_opts), C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_double), C.POINTER(bsm_sign_stats),
                                      C.POINTER(bsm_sign_stats), C.c_void_p]),
    ("bsm_tc2", C.c_int, [C.c_void_p, C.c_double, C.POINTER(bsm_sign_opts),
                          C.POINTER(C.c_void_p), C.POINTER(bsm_tc2_stats), C.c_void_p]),
    ("bsm_trs4", C.c_int, [C.c_void_p, C.c_double, C.POINTER(bsm_sign_opts),
                           C.POINTER(C.c_void_p), C.POINTER(bsm_tc2_stats), C.c_void_p]),
    ("bsm_transpose", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p]),
    ("bsm_submatrix_density", C.c_int, [C.c_void_p, C.c_double, C.POINTER(bsm_sign_opts),
                                        C.POINTER(C.c_void_p), C.POINTER(bsm_sub_stats),
                                        C.c_void_p]),
    ("bsm_density_from_sign", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_double), C.c_void_p]),
    ("bsm_smm_bench", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                C.POINTER(bsm_smm_params), C.c_int32, C.POINTER(C.c_double),
                                C.c_void_p]),
    ("bsm_set_smm_table", C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(bsm_smm_params)]),
    ("bsm_last_error", C.c_char_p, []),
    ("bsm_version", C.c_char_p, []),
    ("bsm_last_smm_kernel", C.c_char_p, []),
]
EXPORTED = [name for name, _, _ in _SIGS]


def load():
    """Load libbsm.so (raises if it is not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is not built; run `python -m "
                                  "paper_2003_03868_amd.build` (no CPU fallback exists)")
            lib = C.CDLL(LIB_PATH)
            for name, res, args in _SIGS:
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def _check(st: int, where: str):
    if st != OK:
        raise BsmError(st, where, load().bsm_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(x):
    """Device or host address of a torch tensor / numpy array (0 if empty)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data if x.size else None
    return x.data_ptr() if x.numel() else None


# ---------------------------------------------------------------- raw API

def bsm_sign_opts_default() -> bsm_sign_opts:
    o = bsm_sign_opts()
    load().bsm_sign_opts_default(C.byref(o))
    return o


def bsm_create(nbrows, nbcols, row_blk_size, col_blk_size, nnzb, row_ptr, col_idx, values,
               on_device, stream=None) -> int:
    h = C.c_void_p()
    rbs = np.ascontiguousarray(row_blk_size, dtype=np.int32)
    cbs = np.ascontiguousarray(col_blk_size, dtype=np.int32)
    st = load().bsm_create(C.byref(h), nbrows, nbcols, _ptr(rbs), _ptr(cbs), nnzb,
                           _ptr(row_ptr), _ptr(col_idx), _ptr(values), int(on_device),
                           _stream(stream))
    _check(st, "bsm_create")
    return h.value


def bsm_destroy(h) -> None:
    _check(load().bsm_destroy(h), "bsm_destroy")


def bsm_get_info(h) -> bsm_info:
    info = bsm_info()
    _check(load().bsm_get_info(h, C.byref(info)), "bsm_get_info")
    return info


def bsm_export(h, row_ptr, col_idx, values, on_device, stream=None) -> None:
    _check(load().bsm_export(h, _ptr(row_ptr), _ptr(col_idx), _ptr(values), int(on_device),
                             _stream(stream)), "bsm_export")


def bsm_multiply(alpha, A, B, beta, Cm, eps_filter=0.0, norm=NORM_FROB, prec=FP64,
                 stream=None) -> bsm_mult_stats:
    stats = bsm_mult_stats()
    st = load().bsm_multiply(float(alpha), A, B, float(beta), Cm, float(eps_filter), int(norm),
                             int(prec), C.byref(stats), _stream(stream))
    _check(st, "bsm_multiply")
    return stats


def bsm_multiply_screened(alpha, A, B, beta, Cm, eps_filter=0.0, norm=NORM_FROB,
                          eps_screen=0.0, stream=None) -> bsm_mult_stats:
    stats = bsm_mult_stats()
    st = load().bsm_multiply_screened(float(alpha), A, B, float(beta), Cm, float(eps_filter),
                                      int(norm), float(eps_screen), C.byref(stats),
                                      _stream(stream))
    _check(st, "bsm_multiply_screened")
    return stats


def bsm_multiply_plan(alpha, A, B, Cm, eps_filter=0.0, norm=NORM_FROB, prec=FP64,
                      stream=None):
    """C = alpha A B and a plan for numeric-only repeats: returns (plan, stats)."""
    plan = C.c_void_p()
    stats = bsm_mult_stats()
    st = load().bsm_multiply_plan(float(alpha), A, B, Cm, float(eps_filter), int(norm), int(prec),
                                  C.byref(plan), C.byref(stats), _stream(stream))
    _check(st, "bsm_multiply_plan")
    return plan.value, stats


def bsm_plan_execute(plan, A, B, Cm, stream=None) -> None:
    _check(load().bsm_plan_execute(plan, A, B, Cm, _stream(stream)), "bsm_plan_execute")


def bsm_plan_status(plan, stream=None) -> int:
    """Bit 0: NaN/Inf; bit 1: the filter would have kept another block set."""
    f = C.c_int32(0)
    _check(load().bsm_plan_status(plan, C.byref(f), _stream(stream)), "bsm_plan_status")
    return f.value


def bsm_plan_destroy(plan) -> None:
    _check(load().bsm_plan_destroy(plan), "bsm_plan_destroy")


def bsm_filter(h, eps_filter, norm=NORM_FROB, stream=None) -> None:
    _check(load().bsm_filter(h, float(eps_filter), int(norm), _stream(stream)), "bsm_filter")


def bsm_block_norms(h, out_dev, stream=None) -> None:
    _check(load().bsm_block_norms(h, _ptr(out_dev), _stream(stream)), "bsm_block_norms")


def bsm_trace(h, stream=None) -> float:
    v = C.c_double()
    _check(load().bsm_trace(h, C.byref(v), _stream(stream)), "bsm_trace")
    return v.value


def bsm_sqdist_identity(h, shift=1.0, stream=None) -> float:
    v = C.c_double()
    _check(load().bsm_sqdist_identity(h, float(shift), C.byref(v), _stream(stream)),
           "bsm_sqdist_identity")
    return v.value


def bsm_sqdist_identity_noalloc(h, shift, out_dev_ptr: int, stream=None) -> int:
    """||A - shift I||_F^2 into the device double at out_dev_ptr (no wait, no
    allocation); returns the status (BsmError is not raised for ECAPACITY)."""
    st = load().bsm_sqdist_identity_noalloc(h, float(shift), C.c_void_p(out_dev_ptr),
                                            _stream(stream))
    if st not in (OK, ECAPACITY):
        _check(st, "bsm_sqdist_identity_noalloc")
    return st


def bsm_inf_norm(h, mu=0.0, stream=None) -> float:
    v = C.c_double()
    _check(load().bsm_inf_norm(h, float(mu), C.byref(v), _stream(stream)), "bsm_inf_norm")
    return v.value


def bsm_shift_scale(h, mu, scale, stream=None) -> int:
    out = C.c_void_p()
    _check(load().bsm_shift_scale(h, float(mu), float(scale), C.byref(out), _stream(stream)),
           "bsm_shift_scale")
    return out.value


def bsm_sign_iterate(h, mu=0.0, opts: bsm_sign_opts | None = None, stream=None):
    """Returns (status, X handle or None, stats).  ENOCONV/ENONFINITE are
    returned, not raised, since the last iterate is still meaningful."""
    out = C.c_void_p()
    stats = bsm_sign_stats()
    o = opts if opts is not None else bsm_sign_opts_default()
    st = load().bsm_sign_iterate(h, float(mu), C.byref(o), C.byref(out), C.byref(stats),
                                 _stream(stream))
    if st not in (OK, ENOCONV, ENONFINITE):
        _check(st, "bsm_sign_iterate")
    return st, out.value, stats


def bsm_mu_bisect(h, n_target, mu_lo, mu_hi, count_tol=0.5, max_steps=40,
                  opts: bsm_sign_opts | None = None, stream=None):
    """Returns (status, mu, X handle or None, stats); ENOCONV is returned,
    not raised, since the last midpoint and its X are still meaningful."""
    out = C.c_void_p()
    mu = C.c_double()
    stats = bsm_mu_stats()
    o = opts if opts is not None else bsm_sign_opts_default()
    st = load().bsm_mu_bisect(h, float(n_target), float(mu_lo), float(mu_hi), float(count_tol),
                              int(max_steps), C.byref(o), C.byref(mu), C.byref(out),
                              C.byref(stats), _stream(stream))
    if st not in (OK, ENOCONV):
        _check(st, "bsm_mu_bisect")
    return st, mu.value, out.value, stats


def bsm_sqrt_inv(s, opts: bsm_sign_opts | None = None, stream=None):
    """Returns (status, S^{1/2} handle, S^{-1/2} handle, stats); ENOCONV is
    returned, not raised (both handles are still set)."""
    a, b = C.c_void_p(), C.c_void_p()
    stats = bsm_sign_stats()
    o = opts if opts is not None else bsm_sign_opts_default()
    st = load().bsm_sqrt_inv(s, C.byref(o), C.byref(a), C.byref(b), C.byref(stats),
                             _stream(stream))
    if st not in (OK, ENOCONV):
        _check(st, "bsm_sqrt_inv")
    return st, a.value, b.value, stats


def bsm_density_nonorth(k, s, mu=0.0, opts: bsm_sign_opts | None = None, stream=None):
    """Returns (status, P handle, trace(P S), sqrt stats, sign stats); ENOCONV
    is returned, not raised."""
    p = C.c_void_p()
    tps = C.c_double()
    s1, s2 = bsm_sign_stats(), bsm_sign_stats()
    o = opts if opts is not None else bsm_sign_opts_default()
    st = load().bsm_density_nonorth(k, s, float(mu), C.byref(o), C.byref(p), C.byref(tps),
                                    C.byref(s1), C.byref(s2), _stream(stream))
    if st not in (OK, ENOCONV):
        _check(st, "bsm_density_nonorth")
    return st, p.value, tps.value, s1, s2


def _purify(name, h, n_occ, opts, stream):
    out = C.c_void_p()
    stats = bsm_tc2_stats()
    o = opts if opts is not None else bsm_sign_opts_default()
    st = getattr(load(), name)(h, float(n_occ), C.byref(o), C.byref(out), C.byref(stats),
                               _stream(stream))
    if st not in (OK, ENOCONV, ENONFINITE):
        _check(st, name)
    return st, out.value, stats


def bsm_tc2(h, n_occ, opts: bsm_sign_opts | None = None, stream=None):
    """Returns (status, P handle or None, stats); ENOCONV/ENONFINITE are
    returned, not raised."""
    return _purify("bsm_tc2", h, n_occ, opts, stream)


def bsm_trs4(h, n_occ, opts: bsm_sign_opts | None = None, stream=None):
    """TRS4 purification; returns (status, P handle or None, stats) as bsm_tc2."""
    return _purify("bsm_trs4", h, n_occ, opts, stream)


def bsm_transpose(a, stream=None) -> int:
    """A^T as a new handle."""
    out = C.c_void_p()
    _check(load().bsm_transpose(a, C.byref(out), _stream(stream)), "bsm_transpose")
    return out.value


def bsm_submatrix_density(h, mu=0.0, opts: bsm_sign_opts | None = None, stream=None):
    """Submatrix-method density; returns (status, P handle or None, stats);
    ENOCONV/ENONFINITE are returned, not raised."""
    out = C.c_void_p()
    stats = bsm_sub_stats()
    o = opts if opts is not None else bsm_sign_opts_default()
    st = load().bsm_submatrix_density(h, float(mu), C.byref(o), C.byref(out), C.byref(stats),
                                      _stream(stream))
    if st not in (OK, ENOCONV, ENONFINITE):
        _check(st, "bsm_submatrix_density")
    return st, out.value, stats


def bsm_add(alpha, a, beta=0.0, b=None, gamma=0.0, eps_filter=0.0, norm=0, stream=None) -> int:
    """C = alpha A + beta B + gamma I, filtered, as a new handle."""
    out = C.c_void_p()
    _check(load().bsm_add(float(alpha), a, float(beta), b, float(gamma), float(eps_filter),
                          int(norm), C.byref(out), _stream(stream)), "bsm_add")
    return out.value


def bsm_density_from_sign(h, stream=None):
    out = C.c_void_p()
    tp = C.c_double()
    _check(load().bsm_density_from_sign(h, C.byref(out), C.byref(tp), _stream(stream)),
           "bsm_density_from_sign")
    return out.value, tp.value


def bsm_smm_bench(m, n, k, n_cblocks, prods_per_cblock, params, reps=3, stream=None):
    """Median kernel ms of every (family, wpg, prefetch) tuple in `params`."""
    arr = (bsm_smm_params * len(params))(*[bsm_smm_params(f, w, p, 0) for f, w, p in params])
    out = (C.c_double * len(params))()
    _check(load().bsm_smm_bench(m, n, k, n_cblocks, prods_per_cblock, len(params), arr, reps,
                                out, _stream(stream)), "bsm_smm_bench")
    return list(out)


def bsm_set_smm_table(entries) -> None:
    """entries: iterable of ((m, n, k), (family, wpg, prefetch)); None clears."""
    if entries is None:
        _check(load().bsm_set_smm_table(-1, None, None), "bsm_set_smm_table")
        return
    entries = list(entries)
    mnk = (C.c_int32 * (3 * len(entries)))(*[v for (t, _) in entries for v in t])
    prm = (bsm_smm_params * len(entries))(*[bsm_smm_params(f, w, p, 0)
                                            for (_, (f, w, p)) in entries])
    _check(load().bsm_set_smm_table(len(entries), mnk, prm), "bsm_set_smm_table")


def bsm_last_error() -> str:
    return load().bsm_last_error().decode()


def bsm_last_smm_kernel() -> str:
    return load().bsm_last_smm_kernel().decode()


def bsm_version() -> str:
    return load().bsm_version().decode()


# --------------------------------------------------------- handle wrapper

class Matrix:
    """Owns a bsm_matrix handle; block sizes are kept for export."""

    def __init__(self, handle: int, row_blk_size, col_blk_size):
        self.handle = handle
        self.row_blk_size = np.ascontiguousarray(row_blk_size, dtype=np.int32)
        self.col_blk_size = np.ascontiguousarray(col_blk_size, dtype=np.int32)

    @classmethod
    def from_arrays(cls, row_blk_size, col_blk_size, row_ptr, col_idx, values,
                    device: bool = True, stream=None) -> "Matrix":
        """Create from host arrays; with device=True they are first staged in
        torch device tensors and handed over as device pointers."""
        rbs = np.ascontiguousarray(row_blk_size, dtype=np.int32)
        cbs = np.ascontiguousarray(col_blk_size, dtype=np.int32)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        va = np.ascontiguousarray(values, dtype=np.float64)
        if device:
            import torch
            rp_d = torch.from_numpy(rp).cuda()
            ci_d = torch.from_numpy(ci).cuda()
            va_d = torch.from_numpy(va).cuda()
            h = bsm_create(rbs.size, cbs.size, rbs, cbs, ci.size, rp_d, ci_d, va_d, 1, stream)
            torch.cuda.current_stream().synchronize()
        else:
            h = bsm_create(rbs.size, cbs.size, rbs, cbs, ci.size, rp, ci, va, 0, stream)
        return cls(h, rbs, cbs)

    @classmethod
    def from_bsr(cls, m, device: bool = True, stream=None) -> "Matrix":
        return cls.from_arrays(m.row_blk_size, m.col_blk_size, m.row_ptr, m.col_idx, m.values,
                               device=device, stream=stream)

    @classmethod
    def empty_like(cls, row_blk_size, col_blk_size, stream=None) -> "Matrix":
        rbs = np.ascontiguousarray(row_blk_size, dtype=np.int32)
        cbs = np.ascontiguousarray(col_blk_size, dtype=np.int32)
        rp = np.zeros(rbs.size + 1, dtype=np.int64)
        h = bsm_create(rbs.size, cbs.size, rbs, cbs, 0, rp, None, None, 0, stream)
        return cls(h, rbs, cbs)

    def info(self) -> bsm_info:
        return bsm_get_info(self.handle)

    def export(self, stream=None):
        """(row_ptr, col_idx, values) as host numpy arrays."""
        inf = self.info()
        rp = np.zeros(inf.nbrows + 1, dtype=np.int64)
        ci = np.zeros(inf.nnzb, dtype=np.int32)
        va = np.zeros(inf.nvalues, dtype=np.float64)
        bsm_export(self.handle, rp, ci, va, 0, stream)
        return rp, ci, va

    def destroy(self):
        if self.handle:
            bsm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.bsm_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
