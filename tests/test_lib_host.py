"""Host side of the GPU library, on the CPU: the library's tree and interaction
lists equal the oracle's bit for bit (two independent codes following the same
rules), the C interface exports every declared symbol, and bad arguments are
rejected before any GPU call."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1209_3516_amd import fmm
from paper_1209_3516_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

TREE_KEYS = ("perm", "keys", "level", "parent", "child_begin", "n_child", "body_begin",
             "n_body", "center", "radius")


def _compare(x, ncrit, theta, leaf_first=False, box=False):
    o = O.OracleFMM(x, ncrit, theta, leaf_first=leaf_first, box_centres=box)
    t = fmm.Tree(x, ncrit, box_centres=box)
    lst = fmm.Lists(t, theta, leaf_first=leaf_first)
    ot, lt = o.tree(), t.view()
    assert lt["n_cells"] == o.num_cells
    for k in TREE_KEYS:
        a, b = np.asarray(ot[k]), np.asarray(lt[k])
        if k == "child_begin":  # leaves: unspecified in the oracle; both use 0
            mask = ot["n_child"] > 0
            a, b = a[mask], b[mask]
        assert a.dtype.kind == b.dtype.kind or k in ("body_begin", "n_body")
        np.testing.assert_array_equal(a, b, err_msg=k)
    for kind in (O.P2P, O.M2L):
        op, oc = o.lists(kind)
        lp, lc = lst.csr(kind)
        np.testing.assert_array_equal(op, lp)
        np.testing.assert_array_equal(oc, lc)
    return o, t, lst


@pytest.mark.parametrize("dist,n,ncrit,theta", [
    ("uniform", 10_000, 64, 0.4), ("uniform", 3000, 1, 0.5), ("uniform", 5000, 8, 0.2),
    ("plummer", 8000, 32, 0.35), ("plummer", 3000, 4, 0.6), ("uniform", 64, 64, 0.4),
    ("uniform", 65, 64, 0.4), ("uniform", 1, 4, 0.4), ("uniform", 2, 1, 0.3)])
@pytest.mark.parametrize("leaf_first", [False, True])
def test_tree_and_lists_match_oracle(dist, n, ncrit, theta, leaf_first):
    x = W.positions(n, dist)
    _compare(x, ncrit, theta, leaf_first)


@pytest.mark.parametrize("dist,n,ncrit,theta", [
    ("uniform", 10_000, 64, 0.4), ("plummer", 8000, 32, 0.35), ("uniform", 3000, 1, 0.5),
    ("uniform", 1, 4, 0.4), ("uniform", 2, 1, 0.3)])
@pytest.mark.parametrize("leaf_first", [False, True])
def test_box_centred_tree_and_lists_match_oracle(dist, n, ncrit, theta, leaf_first):
    x = W.positions(n, dist)
    _compare(x, ncrit, theta, leaf_first, box=True)


def test_box_centred_lists_match_oracle_at_1e6():
    c = W.CONFIGS["plummer-1e6-p6"]
    x = W.positions(c["n"], c["dist"])
    _compare(x, c["ncrit"], c["theta"], box=True)


def test_lists_match_oracle_c1_workload():
    c = W.CONFIGS["uniform-1e4-p4"]
    x = W.positions(c["n"], c["dist"])
    _, _, lst = _compare(x, c["ncrit"], c["theta"])
    s = lst.stats()
    assert s["p2p_entries"] > 0 and s["m2l_entries"] > 0


def test_lists_match_oracle_degenerate_inputs():
    rng = np.random.default_rng(3)
    base = W.uniform_cube(500, seed=41)
    dup = np.concatenate([base, base[:200], base[:50]])          # exact duplicates
    same = np.tile([[0.5, 0.25, 0.125]], (300, 1))               # all coincident
    line = np.stack([np.linspace(0, 1, 700), np.zeros(700), np.zeros(700)], 1)  # flat box
    clustered = np.concatenate([W.uniform_cube(400, seed=42) * 1e-6, W.uniform_cube(400, seed=43)])
    not_f32 = rng.random((800, 3))                                # not FP32-representable
    for x in (dup, same, line, clustered, not_f32):
        for ncrit in (1, 3, 16):
            _compare(x, ncrit, 0.45)


def test_deep_duplicate_leaf_exceeds_ncrit():
    x = np.concatenate([np.tile([[0.3, 0.3, 0.3]], (100, 1)), W.uniform_cube(100, seed=44)])
    _, t, _ = _compare(x, 8, 0.4)
    v = t.view()
    big = (v["n_child"] == 0) & (v["n_body"] > 8)
    assert np.all(v["level"][big] == 21)


def test_fp32_exact_flag():
    assert fmm.Tree(W.uniform_cube(100), 8).view()["fp32_exact"]
    assert not fmm.Tree(np.random.default_rng(0).random((100, 3)), 8).view()["fp32_exact"]


def test_p2p_pair_count():
    x = W.uniform_cube(2000, seed=45)
    t = fmm.Tree(x, 16)
    lst = fmm.Lists(t, 0.4)
    v = t.view()
    ptr, col = lst.csr(fmm.FMM_P2P)
    pairs = 0
    for a in range(len(ptr) - 1):
        for b in col[ptr[a]:ptr[a + 1]]:
            pairs += v["n_body"][a] * v["n_body"][b] - (v["n_body"][a] if a == b else 0)
    assert lst.stats()["p2p_pairs"] == pairs


def test_header_symbols_are_exported():
    hdr = open(os.path.join(ROOT, "include", "fmm.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|size_t|const char \*)\s*(fmm_\w+)\s*\(", hdr,
                              re.M))
    assert declared == set(fmm.EXPORTS)
    L = fmm.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_invalid_arguments_are_rejected_without_gpu():
    L = fmm.lib()
    h = ctypes.c_void_p()
    x = np.ascontiguousarray(W.uniform_cube(10))
    p = x.ctypes.data_as(ctypes.c_void_p)
    assert L.fmm_tree_build(p, 10, 0, ctypes.byref(h)) == fmm.FMM_EINVAL
    assert L.fmm_tree_build(p, -1, 4, ctypes.byref(h)) == fmm.FMM_EINVAL
    bad = x.copy()
    bad[3, 1] = np.nan
    assert L.fmm_tree_build(bad.ctypes.data_as(ctypes.c_void_p), 10, 4,
                            ctypes.byref(h)) == fmm.FMM_EINVAL
    assert b"finite" in L.fmm_last_error()
    bad[3, 1] = np.inf
    assert L.fmm_tree_build(bad.ctypes.data_as(ctypes.c_void_p), 10, 4,
                            ctypes.byref(h)) == fmm.FMM_EINVAL
    t = fmm.Tree(x, 4)
    for theta in (0.0, 1.0, -0.5, float("nan"), 2.0):
        with pytest.raises(fmm.FMMError) as e:
            fmm.Lists(t, theta)
        assert e.value.code == fmm.FMM_EINVAL
    with pytest.raises(fmm.FMMError):
        fmm.Lists(t, 0.4, leaf_first=True).csr(7)
    lst = fmm.Lists(t, 0.4)
    dummy = ctypes.c_void_p(16)
    for p_, prec in ((0, 0), (9, 0), (4, 2)):
        o = fmm._EvalOpts(p_, prec, -1, 0)
        assert L.fmm_evaluate(t._h, lst._h, ctypes.byref(o), dummy, dummy, None,
                              None) == fmm.FMM_EINVAL
    o = fmm._EvalOpts(4, 0, -1, 0)
    assert L.fmm_evaluate(t._h, lst._h, ctypes.byref(o), None, dummy, None,
                          None) == fmm.FMM_EINVAL
    t2 = fmm.Tree(x, 4)
    assert L.fmm_evaluate(t2._h, lst._h, ctypes.byref(o), dummy, dummy, None,
                          None) == fmm.FMM_ESTATE
    assert b"another tree" in L.fmm_last_error()
    # dx without grad_q
    assert L.fmm_evaluate_backward(t._h, lst._h, ctypes.byref(o), dummy, None, dummy, None, None,
                                   dummy, None) == fmm.FMM_EINVAL
    # no w
    assert L.fmm_evaluate_backward(t._h, lst._h, ctypes.byref(o), dummy, dummy, None, dummy,
                                   dummy, dummy, None) == fmm.FMM_EINVAL
    assert L.fmm_last_timings(lst._h, (ctypes.c_double * 8)()) == fmm.FMM_ESTATE
    assert L.fmm_mean_timings(lst._h, 1, (ctypes.c_double * 8)()) == fmm.FMM_ESTATE
    assert L.fmm_mean_timings(lst._h, 0, (ctypes.c_double * 8)()) == fmm.FMM_EINVAL
    assert L.fmm_mean_timings(lst._h, 65, (ctypes.c_double * 8)()) == fmm.FMM_EINVAL
    assert L.fmm_copy_expansions(lst._h, 0, dummy) == fmm.FMM_ESTATE
    # dispatch orders: host lists are not on a device yet; bad kind or len
    n = ctypes.c_int64()
    assert L.fmm_dispatch_order(lst._h, fmm.FMM_P2P, None, 0, ctypes.byref(n)) == fmm.FMM_ESTATE
    assert L.fmm_dispatch_order(lst._h, 7, None, 0, ctypes.byref(n)) == fmm.FMM_EINVAL
    assert L.fmm_dispatch_order(lst._h, fmm.FMM_M2L, None, 0, None) == fmm.FMM_EINVAL
    assert L.fmm_num_terms(0) == -1 and L.fmm_num_terms(4) == 20 and L.fmm_num_terms(8) == 120


def test_noalloc_entry_point_rejects_without_gpu():
    """fmm_evaluate_noalloc checks its arguments before it touches the GPU."""
    L = fmm.lib()
    assert L.fmm_noalloc_scratch_bytes() == 128 << 20
    x = np.ascontiguousarray(W.uniform_cube(300))
    t = fmm.Tree(x, 16)
    lst = fmm.Lists(t, 0.5)
    dummy = ctypes.c_void_p(16)
    for flags in (fmm.FMM_EVAL_TIMING, fmm.FMM_EVAL_KEEP_STAGES, 8):
        o = fmm._EvalOpts(4, 0, -1, flags)
        assert L.fmm_evaluate_noalloc(t._h, lst._h, ctypes.byref(o), dummy, dummy, None,
                                      None) == fmm.FMM_EINVAL
    o = fmm._EvalOpts(4, 0, -1, 0)
    assert L.fmm_evaluate_noalloc(t._h, lst._h, ctypes.byref(o), None, dummy, None,
                                  None) == fmm.FMM_EINVAL
    assert L.fmm_evaluate_noalloc(t._h, lst._h, ctypes.byref(o), dummy, None, None,
                                  None) == fmm.FMM_EINVAL
    assert L.fmm_evaluate_noalloc(fmm.Tree(x, 16)._h, lst._h, ctypes.byref(o), dummy, dummy,
                                  None, None) == fmm.FMM_ESTATE
    hyb = fmm.Lists(t, 0.5, m2p_max=4)
    assert L.fmm_evaluate_noalloc(t._h, hyb._h, ctypes.byref(o), dummy, dummy, None,
                                  None) == fmm.FMM_EINVAL
    assert b"hybrid" in L.fmm_last_error()
    e = fmm.Tree(np.zeros((0, 3)), 4)
    assert L.fmm_evaluate_noalloc(e._h, fmm.Lists(e, 0.4)._h, ctypes.byref(o), None, None, None,
                                  None) == fmm.FMM_OK


def test_empty_tree_evaluation_is_a_noop():
    L = fmm.lib()
    t = fmm.Tree(np.zeros((0, 3)), 4)
    lst = fmm.Lists(t, 0.4)
    o = fmm._EvalOpts(4, 0, -1, 0)
    assert L.fmm_evaluate(t._h, lst._h, ctypes.byref(o), None, None, None, None) == fmm.FMM_OK
    assert lst.csr(fmm.FMM_P2P)[0].tolist() == [0]


def test_term_exponents_cover_total_degree():
    for p in range(1, 9):
        e = fmm.term_exponents(p)
        assert {tuple(r) for r in e.tolist()} == {
            (a, b, c) for a in range(p) for b in range(p) for c in range(p) if a + b + c < p}


def test_lane_layout_table():
    """Lane layouts used by the P2P kernel cover every target with <= 64 lanes."""
    for nt in range(1, 65):
        best = max(((nt * (64 // -(-nt // r))) / (64.0 * r), r) for r in range(1, 9)
                   if -(-nt // r) <= 64)
        assert best[0] >= 0.5 or nt > 32


def test_injected_allocation_failures_return_enomem(monkeypatch):
    x = W.uniform_cube(3000, seed=71)
    ok = fmm.Tree(x, 8)
    tree_fail = lists_fail = 0
    for k in range(1, 8):
        monkeypatch.setenv("FMM_FAULT_INJECT", "alloc:%d" % k)
        try:
            fmm.Tree(x, 8)
        except fmm.FMMError as e:
            assert e.code == fmm.FMM_ENOMEM
            assert b"host memory" in fmm.lib().fmm_last_error()
            tree_fail += 1
        try:
            fmm.Lists(ok, 0.4)
        except fmm.FMMError as e:
            assert e.code == fmm.FMM_ENOMEM
            lists_fail += 1
    monkeypatch.delenv("FMM_FAULT_INJECT")
    assert tree_fail == 4 and lists_fail == 3
    # the library still works afterwards, and gives the same lists
    a, b = fmm.Lists(ok, 0.4), fmm.Lists(fmm.Tree(x, 8), 0.4)
    for kind in (fmm.FMM_P2P, fmm.FMM_M2L):
        np.testing.assert_array_equal(a.csr(kind)[1], b.csr(kind)[1])


def test_log_output(capfd, monkeypatch):
    monkeypatch.setenv("FMM_LOG", "1")
    t = fmm.Tree(W.uniform_cube(500), 16)
    fmm.Lists(t, 0.4)
    err = capfd.readouterr().err
    assert "[fmm] tree: n=500" in err and "[fmm] lists: theta=0.4" in err


def test_plan_too_large_is_refused(monkeypatch):
    """The P2P work plan indexes runs, work items and partial sums with 32-bit
    integers; the traversal refuses lists whose plan would not fit (the limit
    is lowered through the environment to reach that path at a small size)."""
    x = W.uniform_cube(3000, seed=72)
    t = fmm.Tree(x, 16)
    items = fmm.Lists(t, 0.4).stats()["p2p_work_items"]
    assert items > 1
    monkeypatch.setenv("FMM_PLAN_LIMIT", str(items - 1))
    with pytest.raises(fmm.FMMError) as e:
        fmm.Lists(t, 0.4)
    assert e.value.code == fmm.FMM_EINVAL
    assert b"plan too large" in fmm.lib().fmm_last_error()
    monkeypatch.setenv("FMM_PLAN_LIMIT", str(10 ** 12))  # above 2^31 - 1: no effect
    assert fmm.Lists(t, 0.4).stats()["p2p_work_items"] == items


@pytest.mark.parametrize("config,leaf_first", [("uniform-1e6-p4", False),
                                               ("uniform-1e6-p4", True),
                                               ("plummer-1e6-p6", False)])
def test_tree_and_lists_match_oracle_at_benchmark_sizes(config, leaf_first):
    """The headline workload (uniform 10^6, ncrit 64, theta 0.4) in both
    traversal orders and the adaptive one (Plummer 10^6, ncrit 32, theta 0.35):
    tree arrays and both lists equal the oracle's bit for bit."""
    c = W.CONFIGS[config]
    x = W.positions(c["n"], c["dist"])
    _, _, lst = _compare(x, c["ncrit"], c["theta"], leaf_first)
    s = lst.stats()
    print(config, "leaf-first" if leaf_first else "mac-first", s)
    assert s["p2p_entries"] > 0 and s["m2l_entries"] > 0
