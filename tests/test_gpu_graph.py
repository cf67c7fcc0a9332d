"""Sign iterations replayed from captured hipGraphs.

use_graph = 2: pattern-keyed replay of the numeric kernels; use_graph = 1:
device-sized graphs of whole iterations (symbolic phase included) with
fixed-capacity buffers, for uniform block sizes with an FP64 group kernel.
Both run the same kernels on the same data as the normal path, so every
residual r_k and the returned X must match the normal path bit for bit;
against the oracle they are held to the FP64 tolerance.  Each sign call
replays its graphs many times with host waits and eager work (the normal-path
iterations before capture, the trace) in between, and every replay's square
is checked through its residual."""
import numpy as np
import pytest

import synth
from tests.gpu_util import TOL_FP64, TOL_MIXED, assert_same_matrix, from_dev, need_gpu, rel_fro, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _run(h, eps, tol, use_graph, prec=0, fixed=0):
    from paper_2003_03868_amd import bsm
    d = to_dev(h)
    o = bsm.bsm_sign_opts_default()
    o.eps_filter, o.tol, o.prec, o.use_graph, o.fixed_iters = eps, tol, prec, use_graph, fixed
    st, xh, stats = bsm.bsm_sign_iterate(d.handle, 0.0, o)
    x = from_dev(bsm.Matrix(xh, h.row_blk_size, h.col_blk_size)) if xh else None
    return st, x, stats


def _same_run(a, b):
    (st0, x0, s0), (st1, x1, s1) = a, b
    assert st0 == st1
    assert s0.iterations == s1.iterations
    k = s0.iterations + 1
    assert np.array_equal(np.array(s0.r_hist[:k]), np.array(s1.r_hist[:k])), "residuals differ"
    assert list(s0.prec_hist[:k]) == list(s1.prec_hist[:k])
    assert s0.n_multiplies == s1.n_multiplies
    assert s0.n_products == s1.n_products
    assert s0.flops == s1.flops
    assert np.array_equal(x0.row_ptr, x1.row_ptr) and np.array_equal(x0.col_idx, x1.col_idx)
    assert np.array_equal(x0.values, x1.values), "X differs from the normal path"
    assert s0.trace_x == s1.trace_x


GRAPH_CASES = [
    # eps = 0: X fills in after a few updates, then every iteration replays
    dict(n=64, b=5, rc=4.0, eps=0.0, seed=3, tol=1e-10, replays=True, fallbacks=False),
    dict(n=96, b=13, rc=4.5, eps=0.0, seed=4, tol=1e-10, replays=True, fallbacks=False),
    # filtered: the kept pattern settles near convergence, and replayed
    # products whose filter keeps other blocks are re-filtered
    dict(n=200, b=5, rc=6.0, eps=1e-6, seed=5, tol=1e-8, replays=True, fallbacks=True),
    dict(n=100, b=23, rc=4.2, eps=1e-6, seed=6, tol=1e-8, replays=False, fallbacks=True),
    dict(n=160, b=13, rc=5.0, eps=1e-3, seed=11, tol=1e-4, replays=True, fallbacks=True),
]


@pytest.mark.parametrize("c", GRAPH_CASES, ids=lambda c: f"n{c['n']}b{c['b']}e{c['eps']:g}")
def test_graph_replay_matches_normal_path_and_oracle(orc, c):
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(c["n"], c["b"], cutoff=c["rc"], seed=c["seed"])
    ref = _run(h, c["eps"], c["tol"], 0)
    got = _run(h, c["eps"], c["tol"], 2)
    assert got[0] == bsm.OK, bsm.bsm_last_error()
    _same_run(ref, got)
    s = got[2]
    print(f"n={c['n']} b={c['b']} eps={c['eps']:g}: iterations {s.iterations}, "
          f"replays {s.graph_replays}, fallbacks {s.graph_fallbacks}")
    if c["replays"]:
        assert s.graph_replays > 0
    if c["fallbacks"]:
        assert s.graph_fallbacks > 0
    assert ref[2].graph_replays == 0
    x_ref, st_ref, s_ref = orc.sign_ns(h, eps=c["eps"], tol=c["tol"])
    assert s_ref == orc.OK and s.iterations == st_ref["iterations"]
    assert_same_matrix(got[1], x_ref, TOL_FP64, "graph sign")


@pytest.mark.parametrize("mode", [1, 2], ids=["device_sized", "pattern_keyed"])
def test_graph_replay_fixed_iterations(orc, mode):
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=3)
    ref = _run(h, 0.0, 0.0, 0, fixed=12)
    got = _run(h, 0.0, 0.0, mode, fixed=12)
    assert got[0] == bsm.OK and got[2].iterations == 12
    _same_run(ref, got)
    assert got[2].graph_replays > 0
    x_ref, _, _ = orc.sign_ns(h, eps=0.0, fixed_iters=12)
    assert_same_matrix(got[1], x_ref, TOL_FP64, "graph fixed")


@pytest.mark.parametrize("variant", ["3", "4"], ids=["persistent", "class"])
def test_graph_replay_mixed_sizes_and_chunks(orc, monkeypatch, variant):
    """Mixed block sizes (class or persistent kernels) in several chunks."""
    from paper_2003_03868_amd import bsm
    monkeypatch.setenv("BSM_SMM_VARIANT", variant)
    monkeypatch.setenv("BSM_CHUNK_PRODUCTS", "3000")
    h = synth.neighbour_hamiltonian(100, seed=9, cutoff=4.5, size_choices=(5, 13, 23, 26))
    ref = _run(h, 0.0, 1e-9, 0)
    got = _run(h, 0.0, 1e-9, 1)
    assert got[0] == bsm.OK, bsm.bsm_last_error()
    _same_run(ref, got)
    assert got[2].graph_replays > 0
    x_ref, _, _ = orc.sign_ns(h, eps=0.0, tol=1e-9)
    assert_same_matrix(got[1], x_ref, TOL_FP64, "graph mixed")


@pytest.mark.parametrize("mode", [1, 2], ids=["device_sized", "pattern_keyed"])
@pytest.mark.parametrize("prec", [1, 2], ids=["fp32", "split_bf16"])
def test_graph_replay_mixed_precision(orc, prec, mode):
    """Reduced-precision iterations (replayed with mode 2), then FP64 ones
    (device-sized graphs with mode 1)."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 13, cutoff=4.0, seed=12)
    ref = _run(h, 0.0, 1e-9, 0, prec=prec)
    got = _run(h, 0.0, 1e-9, mode, prec=prec)
    assert got[0] == bsm.OK, bsm.bsm_last_error()
    _same_run(ref, got)
    used = list(got[2].prec_hist[:got[2].iterations + 1])
    assert used[0] == prec and used[-1] == bsm.FP64
    x_ref, _, _ = orc.sign_ns(h, eps=0.0, tol=1e-9)
    assert rel_fro(got[1].to_dense(), x_ref.to_dense()) <= TOL_MIXED


# Device-sized graphs (use_graph = 1): every uniform size with a group kernel,
# filtered and unfiltered, and the settled regime of the benchmark workload.
DEV_CASES = [
    dict(n=200, b=5, rc=6.0, eps=1e-6, seed=5, tol=1e-8),
    dict(n=100, b=6, rc=4.5, eps=1e-6, seed=7, tol=1e-8),
    dict(n=160, b=13, rc=5.0, eps=1e-3, seed=11, tol=1e-4),
    dict(n=96, b=13, rc=4.5, eps=0.0, seed=4, tol=1e-10),
    dict(n=100, b=23, rc=4.2, eps=1e-6, seed=6, tol=1e-8),
    dict(n=80, b=26, rc=4.5, eps=1e-6, seed=8, tol=1e-8),
    dict(n=64, b=32, rc=4.0, eps=1e-5, seed=10, tol=1e-8),
    # the benchmark workload's generator and settings at 256 sites (against
    # the normal path only: the oracle's dense-ish products take minutes)
    dict(n=256, b=23, rc=6.0, eps=1e-6, seed=0, tol=1e-6, density=0.1, oracle=False),
]


@pytest.mark.parametrize("c", DEV_CASES, ids=lambda c: f"n{c['n']}b{c['b']}e{c['eps']:g}")
def test_device_sized_graphs_match_normal_path_and_oracle(orc, c):
    from paper_2003_03868_amd import bsm
    kw = dict(density=c["density"]) if "density" in c else {}
    h = synth.neighbour_hamiltonian(c["n"], c["b"], cutoff=c["rc"], seed=c["seed"], **kw)
    print(f"device-sized graphs: n={c['n']} b={c['b']} eps={c['eps']:g}", flush=True)
    ref = _run(h, c["eps"], c["tol"], 0)
    got = _run(h, c["eps"], c["tol"], 1)
    assert got[0] == bsm.OK, bsm.bsm_last_error()
    _same_run(ref, got)
    s = got[2]
    print(f"  iterations {s.iterations}, replays {s.graph_replays}, fallbacks {s.graph_fallbacks}, "
          f"nnzb(X) {list(s.nnzb_x_hist[:s.iterations + 1])}")
    assert s.graph_replays > 0
    assert list(s.nnzb_x_hist[:s.iterations + 1]) == list(ref[2].nnzb_x_hist[:s.iterations + 1])
    assert list(s.nnzb_y_hist[:s.iterations + 1]) == list(ref[2].nnzb_y_hist[:s.iterations + 1])
    if not c.get("oracle", True):
        return
    x_ref, st_ref, s_ref = orc.sign_ns(h, eps=c["eps"], tol=c["tol"])
    assert s_ref == orc.OK and s.iterations == st_ref["iterations"]
    assert_same_matrix(got[1], x_ref, TOL_FP64, "device-sized graph sign")


@pytest.mark.parametrize("eps,chunk", [(0.0, None), (1e-6, None), (1e-6, "3000")],
                         ids=["unfiltered", "filtered", "filtered_chunks"])
def test_device_sized_graphs_mixed_sizes(orc, monkeypatch, eps, chunk):
    """Mixed block sizes {5, 13, 23, 26} with every (m, n) class in one
    persistent launch per multiply (BSM_SMM_VARIANT=7): the graphs run the
    paired-group kernel over the device count of groups, with value offsets
    scanned on the device; the normal path (in chunks of 3000 products when
    asked) gives the same bits."""
    from paper_2003_03868_amd import bsm
    monkeypatch.setenv("BSM_SMM_VARIANT", "7")
    if chunk:
        monkeypatch.setenv("BSM_CHUNK_PRODUCTS", chunk)
    h = synth.neighbour_hamiltonian(120, seed=9, cutoff=4.5, size_choices=(5, 13, 23, 26))
    print(f"mixed sizes, eps {eps:g}, chunk {chunk}", flush=True)
    ref = _run(h, eps, 1e-8, 0)
    got = _run(h, eps, 1e-8, 1)
    assert got[0] == bsm.OK, bsm.bsm_last_error()
    _same_run(ref, got)
    s = got[2]
    print(f"  iterations {s.iterations}, replays {s.graph_replays}, fallbacks {s.graph_fallbacks}, "
          f"nnzb(X) {list(s.nnzb_x_hist[:s.iterations + 1])}")
    assert s.graph_replays > 0
    assert list(s.nnzb_y_hist[:s.iterations + 1]) == list(ref[2].nnzb_y_hist[:s.iterations + 1])
    x_ref, st_ref, s_ref = orc.sign_ns(h, eps=eps, tol=1e-8)
    assert s_ref == orc.OK and s.iterations == st_ref["iterations"]
    assert_same_matrix(got[1], x_ref, TOL_FP64, "device-sized graph sign, mixed sizes")


def test_device_sized_graphs_maxabs_filter(orc):
    """The filter on max |x| per block (BSM_NORM_MAXABS) in the graphs."""
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(200, 5, cutoff=6.0, seed=5)
    runs = []
    for g in (0, 1):
        d = to_dev(h)
        o = bsm.bsm_sign_opts_default()
        o.eps_filter, o.tol, o.norm, o.use_graph = 1e-6, 1e-8, bsm.NORM_MAXABS, g
        st, xh, stats = bsm.bsm_sign_iterate(d.handle, 0.0, o)
        assert st == bsm.OK, bsm.bsm_last_error()
        runs.append((st, from_dev(bsm.Matrix(xh, h.row_blk_size, h.col_blk_size)), stats))
    _same_run(runs[0], runs[1])
    assert runs[1][2].graph_replays > 0
    x_ref, st_ref, s_ref = orc.sign_ns(h, eps=1e-6, tol=1e-8, norm="maxabs")
    assert s_ref == orc.OK and runs[1][2].iterations == st_ref["iterations"]
    assert_same_matrix(runs[1][1], x_ref, TOL_FP64, "device-sized graph sign, max-abs filter")


# BSM_GRAPH_CAPS multiplies the capacities (unfiltered C blocks, groups,
# entries, X, Y): one of them below the sizes makes that buffer overflow.
OVERFLOW_CASES = [
    ("c", "0.5,1,1,1,1", dict(n=200, b=5, rc=6.0, eps=1e-6, seed=5, tol=1e-8)),
    ("groups", "1,0.5,1,1,1", dict(n=200, b=5, rc=6.0, eps=1e-6, seed=5, tol=1e-8)),
    ("entries", "1,1,0.5,1,1", dict(n=96, b=13, rc=4.5, eps=0.0, seed=4, tol=1e-10)),
    ("y", "1,1,1,1,0.5", dict(n=100, b=23, rc=4.2, eps=1e-6, seed=6, tol=1e-8)),
    ("x", "1,1,1,0.01,1", dict(n=100, b=23, rc=4.2, eps=1e-6, seed=6, tol=1e-8)),
    ("mixed_c", "0.5,1,1,1,1", dict(n=120, b=None, rc=4.5, eps=1e-6, seed=9, tol=1e-8)),
    ("mixed_y", "1,1,1,1,0.5", dict(n=120, b=None, rc=4.5, eps=1e-6, seed=9, tol=1e-8)),
]


@pytest.mark.parametrize("which,caps,case", OVERFLOW_CASES, ids=[c[0] for c in OVERFLOW_CASES])
def test_device_sized_graphs_overflow_falls_back(orc, monkeypatch, which, caps, case):
    """A buffer too small for a graph multiply: the overflow is recorded on
    the device, the structure that overflowed is emptied so the later kernels
    do nothing, the multiply's inputs stay intact, and the iteration is redone
    on the normal path; the results stay those of the normal path.  X's
    buffers keep room for the current X only, so an update that grows X
    overflows (the square runs from the graphs, the update is redone)."""
    from paper_2003_03868_amd import bsm
    monkeypatch.setenv("BSM_GRAPH_CAPS", caps)
    if case["b"] is None:
        monkeypatch.setenv("BSM_SMM_VARIANT", "7")
        h = synth.neighbour_hamiltonian(case["n"], seed=case["seed"], cutoff=case["rc"],
                                        size_choices=(5, 13, 23, 26))
    else:
        h = synth.neighbour_hamiltonian(case["n"], case["b"], cutoff=case["rc"], seed=case["seed"])
    print(f"overflow of {which}: n={case['n']} b={case['b']}", flush=True)
    ref = _run(h, case["eps"], case["tol"], 0)
    got = _run(h, case["eps"], case["tol"], 1)
    assert got[0] == bsm.OK, bsm.bsm_last_error()
    _same_run(ref, got)
    s = got[2]
    print(f"  iterations {s.iterations}, replays {s.graph_replays}, fallbacks {s.graph_fallbacks}, "
          f"nnzb(X) {list(s.nnzb_x_hist[:s.iterations + 1])}, "
          f"nnzb(Y) {list(s.nnzb_y_hist[:s.iterations + 1])}")
    assert s.graph_fallbacks > 0
    x_ref, _, _ = orc.sign_ns(h, eps=case["eps"], tol=case["tol"])
    assert_same_matrix(got[1], x_ref, TOL_FP64, f"device-sized graph sign, {which} overflow")


def test_use_graph_value_checked():
    from paper_2003_03868_amd import bsm
    h = synth.neighbour_hamiltonian(64, 5, cutoff=4.0, seed=1)
    with pytest.raises(bsm.BsmError) as e:
        _run(h, 0.0, 1e-8, 3)
    assert e.value.status == bsm.EINVAL
