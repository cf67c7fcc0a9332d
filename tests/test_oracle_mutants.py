"""Plant plausible mistakes in copies of the oracle (on the CPU) and check
that the pins in test_oracle.py catch every one of them."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bsm_oracle.c")

# (name, original text, mutated text): each must occur exactly once.
MUTANTS = [
    ("alpha_sign", "acc[e] *= alpha;", "acc[e] *= -alpha;"),
    ("beta_sign", "acc[e] += beta * cb[e];", "acc[e] -= beta * cb[e];"),
    ("drop_cin_pattern", "mark[cin->col_idx[tc]] = 1;", "(void)tc;"),
    ("filter_threshold", "return !(s < eps * eps);", "return !(s < eps);"),
    ("filter_maxabs", "return !(mx < eps);", "return !(mx <= eps * 0.5);"),
    ("mirrored_b", "acc[r * n + c] += av * bb[t * n + c];",
     "acc[r * n + c] += av * bb[t * n + (n - 1 - c)];"),
    ("a_row_index", "const double av = ab[r * kk + t];", "const double av = ab[(m - 1 - r) * kk + t];"),
    ("ns_coefficient", "orc_multiply_screened(-0.5, x, y, 1.5, x,",
     "orc_multiply_screened(-0.5, x, y, 1.25, x,"),
    ("ns_alpha", "orc_multiply_screened(-0.5, x, y,", "orc_multiply_screened(-0.45, x, y,"),
    ("screen_rule", "block_sq(bb, (int64_t)kk * n) < tau2)", "block_sq(bb, (int64_t)kk * n) < tau)"),
    ("screen_norm", "for (int64_t t = 0; t < len; ++t) s += x[t] * x[t];",
     "for (int64_t t = 0; t < len; ++t) s += fabs(x[t]);"),
    ("o3_coefficient", "orc_shift_scale(y, 1.5, -10.0, &c)", "orc_shift_scale(y, 1.5, -9.0, &c)"),
    ("o3_scale", "orc_multiply(0.125, x, &w,", "orc_multiply(0.25, x, &w,"),
    ("o5_coefficient", "orc_add(35.0, &y2, -180.0, y, 378.0,", "orc_add(35.0, &y2, -180.0, y, 387.0,"),
    ("o5_cin", "orc_shift_scale(y, 0.75, -420.0, &c)", "orc_shift_scale(y, 0.75, -410.0, &c)"),
    ("o5_scale", "orc_multiply(1.0 / 128.0, x, &w,", "orc_multiply(1.0 / 64.0, x, &w,"),
    ("o7_coefficient", "orc_add(231.0, &y3, -1638.0, &y2, -8580.0,", "orc_add(231.0, &y3, -1638.0, &y2, -8508.0,"),
    ("o7_cube", "orc_multiply(1.0, y, &y2, 0.0, NULL, eps, norm_kind, &y3);",
     "orc_multiply(1.0, y, y, 0.0, NULL, eps, norm_kind, &y3);"),
    ("o7_cin", "orc_add(9009.0, &y2, -6006.0, y, 3003.0,", "orc_add(9009.0, &y2, -6006.0, y, 3030.0,"),
    ("o7_scale", "orc_multiply(1.0 / 1024.0, x, &w,", "orc_multiply(1.0 / 512.0, x, &w,"),
    ("sqrt_w_coefficient", "status = orc_shift_scale(&t, 3.0, -0.5, &w);",
     "status = orc_shift_scale(&t, 3.0, -0.45, &w);"),
    ("sqrt_scale", "int s2 = orc_shift_scale(&y, 0.0, sqrt(sc), sqrt_out);",
     "int s2 = orc_shift_scale(&y, 0.0, sc, sqrt_out);"),
    ("isqrt_scale", "s2 = orc_shift_scale(&z, 0.0, 1.0 / sqrt(sc), isqrt_out);",
     "s2 = orc_shift_scale(&z, 0.0, 1.0 / sc, isqrt_out);"),
    ("nonorth_one_sided", "status = orc_multiply(1.0, &k1, &z, 0.0, NULL, eps, norm_kind, &kt);",
     "status = orc_shift_scale(&k1, 0.0, 1.0, &kt);"),
    ("nonorth_back", "s2 = orc_multiply(1.0, &p1, &z, 0.0, NULL, eps, norm_kind, p_out);",
     "s2 = orc_shift_scale(&p1, 0.0, 1.0, p_out);"),
    ("tc2_branch", "if (tx > n_occ) {", "if (tx < n_occ) {"),
    ("tc2_scale", "return orc_shift_scale(h, sc, -0.5 / sc, x);", "return orc_shift_scale(h, sc, -1.0 / sc, x);"),
    ("tc2_update", "return orc_add(2.0, x, -1.0, y, 0.0,", "return orc_add(2.0, x, -0.5, y, 0.0,"),
    ("add_gamma", "tmp[r * m + r] = tmp[r * m + r] + gamma;", "tmp[r * m + r] = tmp[r * m + r] - gamma;"),
    ("add_b_index", "tmp[e] = tmp[e] + beta * b->values[offb[tb] + e];",
     "tmp[e] = tmp[e] + beta * b->values[offb[tb]];"),
    ("residual_norm", "double r = sqrt(orc_sqdist_identity(&y, 1.0)) / n;",
     "double r = sqrt(orc_sqdist_identity(&y, 1.0) / n);"),
    ("shift_sign", "tmp[r * m + r] = scale * (a->values[off[t] + (int64_t)r * m + r] - mu);",
     "tmp[r * m + r] = scale * (a->values[off[t] + (int64_t)r * m + r] + mu);"),
    ("inf_norm_abs", "s += fabs(x[c] - ((j == i && c == r) ? mu : 0.0));",
     "s += (x[c] - ((j == i && c == r) ? mu : 0.0));"),
    ("trs4_f_coefficient", "orc_add(4.0, &x, -3.0, &y, 0.0,", "orc_add(4.0, &x, -2.0, &y, 0.0,"),
    ("trs4_g_operand", "orc_multiply(1.0, &d, &d, 0.0,", "orc_multiply(1.0, &d, &x, 0.0,"),
    ("trs4_gamma_sign", "(n_occ - tf) / tg", "(tf - n_occ) / tg"),
    ("trs4_upper_branch", "if (gamma > 6.0) {", "if (gamma > 2.0) {"),
    ("trs4_no_g", "tg > 0.0 ? (n_occ - tf) / tg : 0.0", "tg > 0.0 ? (n_occ - tf) / tg : 7.0"),
    ("transpose_block", "tmp[c * m + r] = a->values[off[t] + (int64_t)r * n + c];",
     "tmp[r * n + c] = a->values[off[t] + (int64_t)r * n + c];"),
    ("trace_p", "st->trace_p = 0.5 * (n - st->trace_x);", "st->trace_p = 0.5 * (n + st->trace_x);"),
    ("skip_last_k", "for (int64_t ta = a->row_ptr[i]; ta < a->row_ptr[i + 1]; ++ta) {\n                    int32_t k",
     "for (int64_t ta = a->row_ptr[i]; ta + 1 < a->row_ptr[i + 1]; ++ta) {\n                    int32_t k"),
    ("stall_rule", "if (k == max_iter) { status = ORC_ENOCONV; break; }", "if (k == max_iter) { break; }"),
]

# Planted mistakes in the Python submatrix oracle (oracle/submatrix.py).
PY_SRC = os.path.join(ROOT, "oracle", "submatrix.py")
PY_MUTANTS = [
    ("sub_mu_sign", "t -= mu * np.eye(t.shape[0])", "t += mu * np.eye(t.shape[0])"),
    ("sub_eigvec", "x = (v * np.sign(w)) @ v.T", "x = (v * np.sign(w)) @ v"),
    ("sub_half", "pj = 0.5 * (np.eye(t.shape[0]) - x)", "pj = 0.5 * (np.eye(t.shape[0]) + x)"),
    ("sub_column", "out[(int(i), j)] = pj[st[b]:st[b + 1], st[a]:st[a + 1]]",
     "out[(int(i), j)] = pj[st[b]:st[b + 1], 0:st[a + 1] - st[a]]"),
    ("sub_filter", "(blk * blk).sum() < eps * eps", "(blk * blk).sum() < eps"),
    ("sub_missing_block", "            if blk is not None:\n                t[st[a]",
     "            if blk is not None and a != b:\n                t[st[a]"),
]


def _run_py_mutant(tmpdir, name, old, new):
    src = open(PY_SRC).read()
    assert src.count(old) == 1, name
    path = os.path.join(tmpdir, f"m_{name}.py")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    env = dict(os.environ, BSM_ORACLE_SUBMATRIX=path)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-k", "submatrix", os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def _run_mutant(tmpdir, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    msrc = os.path.join(tmpdir, f"m_{name}.c")
    mlib = os.path.join(tmpdir, f"m_{name}.so")
    with open(msrc, "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC",
                           "-shared", "-o", mlib, msrc, "-lm"])
    env = dict(os.environ, BSM_ORACLE_LIB=mlib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_is_caught(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        res = list(ex.map(lambda m: _run_mutant(str(tmp_path), *m), MUTANTS))
        res += list(ex.map(lambda m: _run_py_mutant(str(tmp_path), *m), PY_MUTANTS))
    survivors = [name for name, rc in res if rc == 0]
    assert not survivors, f"pins missed planted mistakes: {survivors}"
