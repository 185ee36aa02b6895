"""GPU parity: the HIP evaluation against the FP64 oracle on identical inputs.

Tolerances (relative L2 over all bodies, potential and gradient separately,
plus a per-body bound of ten times the tolerance, see tests/bounds.py):
  * FP64 mode vs oracle: 1e-12 (same method, different summation order);
  * mixed mode (FP32 P2P/M2L with Kahan-compensated P2P sums) vs oracle:
    1e-5 for p <= 6, 3e-5 for p = 8.
Interaction lists are compared bit for bit on the CPU (test_lib_host.py).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from tests.bounds import assert_close, rel  # noqa: E402
from paper_1209_3516_amd import fmm  # noqa: E402
from paper_1209_3516_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu_eval(x, q, ncrit, theta, p, precision, leaf_first=False, **kw):
    t = fmm.Tree(x, ncrit)
    lst = fmm.Lists(t, theta, leaf_first=leaf_first)
    dt = torch.float64 if precision == "fp64" else torch.float32
    qt = torch.tensor(q, dtype=dt, device=DEV)
    phi, g = fmm.evaluate(t, lst, qt, p, precision, **kw)
    torch.cuda.synchronize()
    return t, lst, phi.double().cpu().numpy(), g.double().cpu().numpy()


def tol(precision, p):
    if precision == "fp64":
        return 1e-12
    return 3e-5 if p >= 8 else 1e-5


CASES = [
    # name, dist, n, charges, ncrit, theta, p
    ("c1-uniform-1e4", "uniform", 10_000, "signed", 64, 0.4, 4),
    ("plummer-6000", "plummer", 6_000, "positive", 32, 0.35, 6),
    ("uniform-3000-p8", "uniform", 3_000, "signed", 8, 0.3, 8),
    ("uniform-2000-p1", "uniform", 2_000, "signed", 16, 0.5, 1),
    ("uniform-2500-p3", "uniform", 2_500, "signed", 5, 0.6, 3),
    ("plummer-4000-p5", "plummer", 4_000, "signed", 12, 0.45, 5),
    ("uniform-3000-p7", "uniform", 3_000, "signed", 10, 0.35, 7),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_full_evaluation_matches_oracle(case, precision):
    name, dist, n, ch, ncrit, theta, p = case
    print("case", name, precision, flush=True)
    x = W.positions(n, dist)
    q = W.charges(n, ch)
    ref = O.OracleFMM(x, ncrit, theta).evaluate(q, p)
    _, _, phi, g = gpu_eval(x, q, ncrit, theta, p, precision)
    assert_close(phi, ref["phi"], tol(precision, p), "phi")
    assert_close(g, ref["grad"], tol(precision, p), "grad")


def test_leaf_first_lists():
    x = W.uniform_cube(3000, seed=9)
    q = W.charges(3000, seed=10)
    ref = O.OracleFMM(x, 16, 0.4, leaf_first=True).evaluate(q, 4)
    for prec in ("fp64", "mixed"):
        _, _, phi, g = gpu_eval(x, q, 16, 0.4, 4, prec, leaf_first=True)
        assert_close(phi, ref["phi"], tol(prec, 4), "phi")
        assert_close(g, ref["grad"], tol(prec, 4), "grad")


@pytest.mark.parametrize("p", [2, 4, 5, 6, 7, 8])
def test_staged_expansions_match_oracle(p):
    """Multipoles after the upward pass, locals after M2L and after L2L (FP64)."""
    x = W.plummer(3000, seed=12)
    q = W.charges(3000, seed=13)
    o = O.OracleFMM(x, 10, 0.5)
    ref = o.evaluate(q, p, staged=True)
    t, lst, phi, g = gpu_eval(x, q, 10, 0.5, p, "fp64", keep_stages=True)
    ex_lib = [tuple(r) for r in fmm.term_exponents(p).tolist()]
    ex_or = [tuple(r) for r in O.term_exponents(p).tolist()]
    perm = [ex_lib.index(e) for e in ex_or]  # oracle term k -> library column
    for kind, key in ((0, "M"), (1, "L_m2l"), (2, "L")):
        got = fmm.copy_expansions(lst, kind, p)[:, perm]
        want = ref[key]
        scale = np.max(np.abs(want), axis=1, keepdims=True) + 1e-300
        assert np.max(np.abs(got - want) / scale) <= 1e-11, key


@pytest.mark.parametrize("p", [4, 6, 8])
def test_staged_expansions_match_oracle_mixed(p):
    """The FP32 path's multipoles after the upward pass, locals after M2L and
    after L2L, row by row against the FP64 oracle (relative to each row's
    largest term): the staged values the mixed-precision kernels produce, not
    only their effect on the final norms."""
    x = W.plummer(6000, seed=12)
    q = W.charges(6000, seed=13)
    o = O.OracleFMM(x, 16, 0.45)
    ref = o.evaluate(q, p, staged=True)
    t, lst, phi, g = gpu_eval(x, q, 16, 0.45, p, "mixed", keep_stages=True)
    ex_lib = [tuple(r) for r in fmm.term_exponents(p).tolist()]
    ex_or = [tuple(r) for r in O.term_exponents(p).tolist()]
    perm = [ex_lib.index(e) for e in ex_or]
    for kind, key, worst in ((0, "M", 1e-5), (1, "L_m2l", 1e-4), (2, "L", 1e-4)):
        got = fmm.copy_expansions(lst, kind, p)[:, perm]
        want = ref[key]
        scale = np.max(np.abs(want), axis=1) + 1e-300
        err = np.max(np.abs(got - want), axis=1) / scale
        assert np.max(err) <= worst, (key, float(np.max(err)))
        assert np.median(err) <= 3e-6, (key, float(np.median(err)))


def test_fp64_top_levels_p8():
    """Mixed mode with the top three levels kept in FP64 (p >= 8)."""
    x = W.uniform_cube(20_000, seed=14)
    q = W.charges(20_000, seed=15)
    ref = O.OracleFMM(x, 32, 0.3).evaluate(q, 8)
    for top in (-1, -2, 5):
        _, _, phi, g = gpu_eval(x, q, 32, 0.3, 8, "mixed", fp64_top_levels=top)
        assert_close(phi, ref["phi"], 3e-5, "phi top=%d" % top)
        assert_close(g, ref["grad"], 3e-5, "grad top=%d" % top)


EDGE = [
    ("single-body", np.array([[0.1, 0.2, 0.3]]), 4),
    ("two-bodies", np.array([[0.0, 0.0, 0.0], [1.0, 0.5, 0.25]]), 1),
    ("one-leaf", None, 64),
    ("all-coincident", np.tile([[0.25, 0.5, 0.75]], (100, 1)), 8),
    ("duplicates", "dup", 4),
    ("deep-big-leaf", "deep", 8),
    ("big-leaf-small-tail", "tail", 8),
    ("not-fp32", "rand", 16),
    ("flat-line", "line", 4),
]


def _edge_points(spec):
    if spec is None:
        return W.uniform_cube(50, seed=16)
    if isinstance(spec, np.ndarray):
        return spec
    if spec == "dup":
        b = W.uniform_cube(400, seed=17)
        return np.concatenate([b, b[:150], b[:40]])
    if spec == "deep":  # 300 coincident bodies: a level-21 leaf, several target groups
        return np.concatenate([np.tile([[0.3, 0.3, 0.3]], (300, 1)), W.uniform_cube(700, seed=18)])
    if spec == "tail":  # a level-21 leaf of 70 bodies: target groups of 64 and 6, the
        # last one on one lane per source stream, with 70 self sources
        return np.concatenate([np.tile([[0.6, 0.2, 0.4]], (70, 1)), W.uniform_cube(500, seed=25)])
    if spec == "rand":
        return np.random.default_rng(19).random((2000, 3))
    if spec == "line":  # canonical (FP32-representable) points on a segment
        line = np.stack([np.linspace(0, 1, 900), np.zeros(900), np.full(900, 0.5)], 1)
        return line.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,spec,ncrit", EDGE, ids=[e[0] for e in EDGE])
def test_edge_cases(name, spec, ncrit, precision):
    print("edge", name, precision, flush=True)
    x = _edge_points(spec)
    q = W.charges(x.shape[0], seed=20)
    ref = O.OracleFMM(x, ncrit, 0.4).evaluate(q, 4)
    _, _, phi, g = gpu_eval(x, q, ncrit, 0.4, 4, precision)
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(g))
    if np.linalg.norm(ref["phi"]) == 0:
        assert np.all(phi == 0) and np.all(g == 0)
        return
    assert_close(phi, ref["phi"], tol(precision, 4), "phi")
    assert_close(g, ref["grad"], tol(precision, 4), "grad")


def test_long_rows_are_chunked():
    """Leaves of ~2000 bodies: rows of >8192 sources (several chunks) and >64
    targets per leaf (several target groups)."""
    x = W.uniform_cube(30_000, seed=21)
    q = W.charges(30_000, seed=22)
    ref = O.OracleFMM(x, 2000, 0.4).evaluate(q, 4)
    for prec in ("fp64", "mixed"):
        _, lst, phi, g = gpu_eval(x, q, 2000, 0.4, 4, prec)
        assert lst.stats()["p2p_max_row_sources"] > 8192
        assert_close(phi, ref["phi"], tol(prec, 4), "phi")
        assert_close(g, ref["grad"], tol(prec, 4), "grad")


def max_run_starts_per_batch(t, lst, batch=384):
    """The most starts of source runs among the positions of one staged batch
    of 384 sources in any P2P row (entries of consecutive leaves whose bodies
    follow each other in memory form one run; the leaf itself is not a run)."""
    v = t.view()
    ptr, col = lst.csr(fmm.FMM_P2P)
    nb, bb = v["n_body"], v["body_begin"]
    best = 0
    for a in np.flatnonzero(v["n_child"] == 0):
        c = col[ptr[a]:ptr[a + 1]]
        c = c[c != a]
        if c.size == 0:
            continue
        new = np.ones(c.size, bool)
        new[1:] = bb[c[1:]] != bb[c[:-1]] + nb[c[:-1]]
        pos = np.concatenate([[0], np.cumsum(nb[c])[:-1]])[new]
        best = max(best, int(np.bincount(pos // batch).max()))
    return best


def test_many_run_starts_per_batch():
    """Leaves of at most 4 bodies on a Plummer sphere at theta = 0.25: more than
    64 runs start inside one staged batch, so the staging flags the run starts
    in more than one round of 64 lanes."""
    x = W.plummer(5000, seed=27)
    q = W.charges(5000, seed=28)
    t = fmm.Tree(x, 4)
    lst = fmm.Lists(t, 0.25)
    assert max_run_starts_per_batch(t, lst) > 64
    ref = O.OracleFMM(x, 4, 0.25).evaluate(q, 4)
    for prec in ("fp64", "mixed"):
        _, _, phi, g = gpu_eval(x, q, 4, 0.25, 4, prec)
        assert_close(phi, ref["phi"], tol(prec, 4), "phi")
        assert_close(g, ref["grad"], tol(prec, 4), "grad")


def test_repeat_is_bitwise_identical():
    x = W.plummer(20_000, seed=23)
    q = W.charges(20_000, seed=24)
    t = fmm.Tree(x, 32)
    lst = fmm.Lists(t, 0.35)
    qt = torch.tensor(q, dtype=torch.float32, device=DEV)
    a = fmm.evaluate(t, lst, qt, 6)
    b = fmm.evaluate(t, lst, qt, 6)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_switching_order_and_precision_on_one_lists():
    x = W.uniform_cube(5000, seed=25)
    q = W.charges(5000, seed=26)
    o = O.OracleFMM(x, 32, 0.4)
    t = fmm.Tree(x, 32)
    lst = fmm.Lists(t, 0.4)
    for p, prec in ((4, "mixed"), (6, "fp64"), (3, "mixed"), (4, "fp64")):
        dt = torch.float64 if prec == "fp64" else torch.float32
        phi, g = fmm.evaluate(t, lst, torch.tensor(q, dtype=dt, device=DEV), p, prec)
        ref = o.evaluate(q, p)
        assert_close(phi.double().cpu().numpy(), ref["phi"], tol(prec, p), "phi")
        assert_close(g.double().cpu().numpy(), ref["grad"], tol(prec, p), "grad")


def test_direct_sum_kernel_matches_oracle():
    x = W.uniform_cube(20_000, seed=27)
    q = W.charges(20_000, seed=28)
    tg = W.sample_targets(20_000, 300)
    phi, g = fmm.direct(torch.tensor(x, device=DEV), torch.tensor(q, device=DEV),
                        torch.tensor(tg, device=DEV))
    rphi, rg = O.direct(x, q, tg)
    assert_close(phi.cpu().numpy(), rphi, 1e-13, "phi")
    assert_close(g.cpu().numpy(), rg, 1e-13, "grad")


def test_timings_are_reported():
    x = W.uniform_cube(20_000, seed=29)
    t = fmm.Tree(x, 64)
    lst = fmm.Lists(t, 0.4)
    qt = torch.tensor(W.charges(20_000), dtype=torch.float32, device=DEV)
    fmm.evaluate(t, lst, qt, 4, timing=True, serial=True)
    ms = fmm.last_timings(lst)
    assert ms["total"] > 0 and ms["p2p"] > 0
    # serial: the phases tile the total up to the cost of the event records
    covered = sum(ms[k] for k in fmm.PHASES[:-1])
    assert covered <= ms["total"] + 1e-3 and covered >= ms["total"] - 0.02
    fmm.evaluate(t, lst, qt, 4, timing=True)  # overlapped: phases overlap the total
    ms = fmm.last_timings(lst)
    assert 0 < ms["p2p"] <= ms["total"] and ms["m2l"] > 0


def test_mean_timings_over_a_run_without_waits():
    """fmm_mean_timings: the mean of the per-evaluation times of the last n
    timed evaluations (the same events fmm_last_timings reads one by one); an
    untimed evaluation starts the count again; the allocation-free entry
    point leaves the timings of the last timed fmm_evaluate as they are."""
    x = W.uniform_cube(20_000, seed=29)
    t = fmm.Tree(x, 64)
    lst = fmm.Lists(t, 0.4)
    qt = torch.tensor(W.charges(20_000), dtype=torch.float32, device=DEV)
    one = []
    for _ in range(3):
        fmm.evaluate(t, lst, qt, 4, timing=True)
        one.append(fmm.last_timings(lst))
    mean = fmm.mean_timings(lst, 3)
    for k in fmm.PHASES:
        assert abs(mean[k] - sum(o[k] for o in one) / 3) <= 1e-9 * max(1.0, abs(mean[k]))
    assert fmm.mean_timings(lst, 1)["total"] == one[-1]["total"]
    with pytest.raises(fmm.FMMError) as e:
        fmm.mean_timings(lst, 4)
    assert e.value.code == fmm.FMM_ESTATE
    with pytest.raises(fmm.FMMError) as e:
        fmm.mean_timings(lst, fmm.TIMING_HISTORY + 1)
    assert e.value.code == fmm.FMM_EINVAL
    # a run longer than the history: the newest TIMING_HISTORY are held
    for _ in range(fmm.TIMING_HISTORY + 2):
        fmm.evaluate(t, lst, qt, 4, timing=True)
    assert fmm.mean_timings(lst, fmm.TIMING_HISTORY)["p2p"] > 0
    phi = torch.empty(20_000, dtype=torch.float32, device=DEV)
    g = torch.empty(20_000, 3, dtype=torch.float32, device=DEV)
    fmm.evaluate_noalloc(t, lst, qt, phi, g, 4)
    torch.cuda.synchronize()
    assert fmm.mean_timings(lst, 2)["total"] > 0
    fmm.evaluate(t, lst, qt, 4)  # untimed: nothing timed is held any more
    with pytest.raises(fmm.FMMError) as e:
        fmm.mean_timings(lst, 1)
    assert e.value.code == fmm.FMM_ESTATE


def test_serial_and_overlapped_agree_bitwise():
    x = W.uniform_cube(50_000, seed=31)
    t = fmm.Tree(x, 64)
    lst = fmm.Lists(t, 0.4)
    qt = torch.tensor(W.charges(50_000), dtype=torch.float32, device=DEV)
    a = fmm.evaluate(t, lst, qt, 4, serial=True)
    b = fmm.evaluate(t, lst, qt, 4)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
