"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* derivatives of 1/r: textbook closed forms (|m| <= 3), central finite
  differences, and harmonicity (the Laplacian of 1/r vanishes away from 0);
* M2L and harmonicity: the local coefficients of one M2L are trace-free
  (L_{k+2e_x} + L_{k+2e_y} + L_{k+2e_z} = 0), and a multipole whose terms with
  n_z >= 2 are moved onto lower z (M_n -> -M at n-2e_z+2e_x and n-2e_z+2e_y)
  has the same M2L, both exactly under the |n| + |k| <= p-1 truncation;
* translations: M2M and L2L are exact re-centrings of polynomials, so
  M2M(P2M about the child) == P2M about the parent and L2P(L2L(L)) == L2P(L);
* single-source exactness and the monopole case p = 1;
* M2L convergence: error of an accepted pair falls like ((a+b)/R)^p
  (section 3.2 states the theta^p error bound);
* full FMM: N <= ncrit and theta -> 0 reduce to the O(N^2) direct sum; the
  error against the direct sum falls monotonically with p; the far-field
  operator is symmetric (w . phi[q] == q . phi[w]).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1209_3516_amd import workloads as W


def _axes(m):
    out = []
    for d in range(3):
        out += [d] * int(m[d])
    return out


def _closed_form(m, R):
    """D^m (1/|R|) for |m| <= 3, from the textbook formulas."""
    r2 = float(R @ R)
    r = math.sqrt(r2)
    ax = _axes(m)
    dl = lambda i, j: 1.0 if i == j else 0.0  # noqa: E731
    if len(ax) == 0:
        return 1.0 / r
    if len(ax) == 1:
        return -R[ax[0]] / r ** 3
    if len(ax) == 2:
        i, j = ax
        return (3.0 * R[i] * R[j] - dl(i, j) * r2) / r ** 5
    i, j, k = ax
    return (-15.0 * R[i] * R[j] * R[k] / r ** 7
            + 3.0 * (dl(i, j) * R[k] + dl(i, k) * R[j] + dl(j, k) * R[i]) / r ** 5)


def test_term_set_is_total_degree_below_p():
    for p in range(1, 10):
        ex = O.term_exponents(p)
        assert ex.shape[0] == p * (p + 1) * (p + 2) // 6
        want = {m for m in itertools.product(range(p), repeat=3) if sum(m) <= p - 1}
        assert {tuple(int(v) for v in m) for m in ex} == want


@pytest.mark.parametrize("R", [(1.0, 2.0, 2.0), (0.3, -0.7, 0.2), (-1e-3, 2e-3, 5e-4)])
def test_derivatives_closed_forms(R):
    R = np.array(R)
    p = 4
    D = O.derivatives(p, R)
    for t, m in enumerate(O.term_exponents(p)):
        want = _closed_form(m, R)
        assert D[t] == pytest.approx(want, rel=1e-13, abs=1e-13 * abs(_closed_form((0, 0, 0), R)))


def test_derivatives_exact_rational_point():
    # R = (1, 2, 2), |R| = 3: D^(1,1,0) = 3*1*2/3^5 = 6/243, D^(2,0,0) = (3 - 9)/243
    D = O.derivatives(3, np.array([1.0, 2.0, 2.0]))
    ex = [tuple(m) for m in O.term_exponents(3)]
    assert D[ex.index((0, 0, 0))] == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert D[ex.index((1, 0, 0))] == pytest.approx(-1.0 / 27.0, rel=1e-15)
    assert D[ex.index((1, 1, 0))] == pytest.approx(6.0 / 243.0, rel=1e-15)
    assert D[ex.index((2, 0, 0))] == pytest.approx(-6.0 / 243.0, rel=1e-15)


@pytest.mark.parametrize("p", [4, 8, 10])
def test_derivatives_finite_differences(p):
    rng = np.random.default_rng(11)
    ex = [tuple(int(v) for v in m) for m in O.term_exponents(p)]
    for _ in range(3):
        R = rng.uniform(-1, 1, 3) + np.array([1.5, 0.0, 0.0])
        h = 1e-5
        D = O.derivatives(p, R)
        for t, m in enumerate(ex):
            if sum(m) == 0:
                continue
            d = int(np.argmax(m))
            lower = list(m)
            lower[d] -= 1
            e = np.zeros(3)
            e[d] = h
            s = ex.index(tuple(lower))
            fd = (O.derivatives(p, R + e)[s] - O.derivatives(p, R - e)[s]) / (2 * h)
            scale = math.factorial(sum(m)) / np.linalg.norm(R) ** (sum(m) + 1)
            assert abs(fd - D[t]) <= 1e-6 * scale, (m, fd, D[t])


@pytest.mark.parametrize("p", [3, 6, 9])
def test_derivatives_harmonic(p):
    rng = np.random.default_rng(12)
    ex = [tuple(int(v) for v in m) for m in O.term_exponents(p)]
    for _ in range(5):
        R = rng.uniform(-2, 2, 3)
        D = O.derivatives(p, R)
        for m in ex:
            if sum(m) > p - 3:
                continue
            lap = 0.0
            for d in range(3):
                mm = list(m)
                mm[d] += 2
                lap += D[ex.index(tuple(mm))]
            scale = math.factorial(sum(m) + 2) / np.linalg.norm(R) ** (sum(m) + 3)
            assert abs(lap) <= 1e-12 * scale


@pytest.mark.parametrize("p", [3, 4, 6, 8])
def test_m2l_harmonic_identities(p):
    # Both identities keep the degree of the index they act on, so the
    # truncation |n| + |k| <= p-1 cuts every term of them at the same place.
    rng = np.random.default_rng(40 + p)
    ex = [tuple(int(v) for v in m) for m in O.term_exponents(p)]
    idx = {m: i for i, m in enumerate(ex)}
    for _ in range(4):
        XB = rng.uniform(-0.5, 0.5, 3)
        XA = XB + rng.normal(size=3) * 2.0
        M = rng.normal(size=len(ex))
        L = O.m2l(p, XA, XB, M)
        # trace-free locals
        for k in ex:
            if sum(k) > p - 3:
                continue
            terms = [L[idx[(k[0] + 2 * (d == 0), k[1] + 2 * (d == 1), k[2] + 2 * (d == 2))]]
                     for d in range(3)]
            assert abs(sum(terms)) <= 1e-12 * sum(abs(t) for t in terms) + 1e-300
        # fold the z exponent of the multipole down to 0 or 1, one step at a time
        F = M.copy()
        for m in sorted(ex, key=lambda m: -m[2]):
            if m[2] < 2:
                continue
            F[idx[(m[0] + 2, m[1], m[2] - 2)]] -= F[idx[m]]
            F[idx[(m[0], m[1] + 2, m[2] - 2)]] -= F[idx[m]]
            F[idx[m]] = 0.0
        assert all(F[idx[m]] == 0.0 for m in ex if m[2] >= 2)
        LF = O.m2l(p, XA, XB, F)
        np.testing.assert_allclose(LF, L, rtol=0, atol=1e-11 * np.abs(L).max())
        # and a multipole with terms of z exponent >= 2 does change M2L if they
        # are simply dropped (the identity is not vacuous)
        if p >= 3:
            Z = M.copy()
            for m in ex:
                if m[2] >= 2:
                    Z[idx[m]] = 0.0
            assert np.abs(O.m2l(p, XA, XB, Z) - L).max() > 1e-6 * np.abs(L).max()


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
def test_m2m_reproduces_p2m_about_parent(p):
    rng = np.random.default_rng(13)
    Xc = rng.uniform(0, 1, 3)
    XP = Xc + rng.uniform(-0.3, 0.3, 3)
    xyz = Xc + rng.uniform(-0.1, 0.1, (20, 3))
    q = rng.uniform(-1, 1, 20)
    Mc = O.p2m(p, Xc, xyz, q)
    MP = O.m2m(p, XP, Xc, Mc)
    want = O.p2m(p, XP, xyz, q)
    assert np.max(np.abs(MP - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
def test_l2l_is_exact_recentring(p):
    rng = np.random.default_rng(14)
    T = O.num_terms(p)
    LP = rng.standard_normal(T)
    XP = rng.uniform(0, 1, 3)
    Xc = XP + rng.uniform(-0.2, 0.2, 3)
    y = Xc + rng.uniform(-0.1, 0.1, (10, 3))
    Lc = O.l2l(p, XP, Xc, LP)
    f1, g1 = O.l2p(p, Xc, Lc, y)
    f0, g0 = O.l2p(p, XP, LP, y)
    assert np.max(np.abs(f1 - f0)) <= 1e-12 * np.max(np.abs(f0))
    assert np.max(np.abs(g1 - g0)) <= 1e-12 * np.max(np.abs(g0))


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_single_source_is_exact(p):
    XB = np.array([0.1, 0.2, 0.3])
    XA = np.array([1.4, -0.5, 0.9])
    q = 0.7
    M = O.p2m(p, XB, XB[None, :], np.array([q]))
    L = O.m2l(p, XA, XB, M)
    f, g = O.l2p(p, XA, L, XA[None, :])
    R = XA - XB
    r = np.linalg.norm(R)
    assert f[0] == pytest.approx(q / r, rel=1e-15)
    want_g = q * (XB - XA) / r ** 3 if p >= 2 else np.zeros(3)
    np.testing.assert_allclose(g[0], want_g, rtol=1e-14, atol=1e-16)


def test_monopole_p1():
    rng = np.random.default_rng(15)
    XB = np.zeros(3)
    xyz = rng.uniform(-0.1, 0.1, (30, 3))
    q = rng.uniform(-1, 1, 30)
    XA = np.array([2.0, 1.0, -1.0])
    L = O.m2l(1, XA, XB, O.p2m(1, XB, xyz, q))
    f, g = O.l2p(1, XA, L, XA[None, :])
    assert f[0] == pytest.approx(q.sum() / np.linalg.norm(XA), rel=1e-14)
    assert np.all(g == 0.0)


def test_m2l_error_falls_like_ratio_to_the_p():
    rng = np.random.default_rng(16)
    a = b = 0.15
    XB = np.zeros(3)
    XA = np.array([1.0, 0.0, 0.0])
    src = XB + b * rng.uniform(-1, 1, (40, 3)) / math.sqrt(3)
    q = rng.uniform(-1, 1, 40)
    tgt = XA + a * rng.uniform(-1, 1, (20, 3)) / math.sqrt(3)
    R = 1.0
    rho = (a + b) / R
    dphi = np.array([np.sum(q / np.linalg.norm(src - y, axis=1)) for y in tgt])
    errs = []
    for p in range(1, 11):
        L = O.m2l(p, XA, XB, O.p2m(p, XB, src, q))
        f, _ = O.l2p(p, XA, L, tgt)
        err = np.max(np.abs(f - dphi))
        errs.append(err)
        assert err <= np.sum(np.abs(q)) / (R - a - b) * rho ** p
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_fmm_single_leaf_is_direct_sum():
    x = W.uniform_cube(50)
    q = W.charges(50)
    o = O.OracleFMM(x, 64, 0.4)
    assert o.num_cells == 1
    r = o.evaluate(q, 4)
    dphi, dg = O.direct(x, q)
    assert _rel(r["phi"], dphi) < 1e-14
    assert _rel(r["grad"], dg) < 1e-14


def test_fmm_tiny_theta_is_direct_sum():
    x = W.uniform_cube(600, seed=7)
    q = W.charges(600, seed=8)
    o = O.OracleFMM(x, 4, 1e-6)
    mptr, mcol = o.lists(O.M2L)
    t = o.tree()
    assert len(mcol) > 0  # single-body leaves still meet the MAC, and are exact
    rows = np.repeat(np.arange(o.num_cells), np.diff(mptr))
    assert np.all(t["radius"][rows] == 0) and np.all(t["radius"][mcol] == 0)
    r = o.evaluate(q, 3)
    dphi, dg = O.direct(x, q)
    assert _rel(r["phi"], dphi) < 1e-13
    assert _rel(r["grad"], dg) < 1e-13


@pytest.mark.parametrize("dist,theta", [("uniform", 0.4), ("uniform", 0.6), ("plummer", 0.35)])
def test_fmm_error_falls_with_p(dist, theta):
    n = 4000
    x = W.positions(n, dist)
    q = W.charges(n)
    o = O.OracleFMM(x, 16, theta)
    dphi, dg = O.direct(x, q)
    ep, eg = [], []
    for p in range(1, 9):
        r = o.evaluate(q, p)
        ep.append(_rel(r["phi"], dphi))
        eg.append(_rel(r["grad"], dg))
    assert all(ep[i + 1] < ep[i] for i in range(7)), ep
    assert all(eg[i + 1] < eg[i] for i in range(7)), eg
    # the per-pair bound falls as theta^p, so seven more orders gain at least theta^7
    assert ep[-1] / ep[0] < theta ** 7
    assert eg[-1] / eg[0] < theta ** 6


def test_fmm_c1_workload_accuracy():
    n = 10_000
    x = W.uniform_cube(n)
    q = W.charges(n)
    o = O.OracleFMM(x, 64, 0.4)
    r = o.evaluate(q, 4)
    dphi, dg = O.direct(x, q)
    assert _rel(r["phi"], dphi) < 2e-3
    assert _rel(r["grad"], dg) < 5e-4


@pytest.mark.parametrize("leaf_first", [False, True])
def test_fmm_operator_is_symmetric(leaf_first):
    n = 3000
    x = W.uniform_cube(n, seed=21)
    q = W.charges(n, seed=22)
    w = W.weights(n, seed=23)
    o = O.OracleFMM(x, 8, 0.5, leaf_first=leaf_first)
    for p in (2, 4, 7):
        a = w @ o.evaluate(q, p)["phi"]
        b = q @ o.evaluate(w, p)["phi"]
        assert a == pytest.approx(b, rel=1e-12)


def test_fmm_coincident_bodies():
    x = W.uniform_cube(300, seed=31)
    x = np.concatenate([x, x[:100], x[:20]])  # exact duplicates
    q = W.charges(x.shape[0], seed=32)
    dphi, dg = O.direct(x, q)
    for ncrit in (1, 4, 64):
        # theta -> 0: only exact interactions remain, so the direct sum (zero
        # distance skipped) is reproduced to rounding
        r = O.OracleFMM(x, ncrit, 1e-6).evaluate(q, 3)
        assert _rel(r["phi"], dphi) < 1e-13
        assert _rel(r["grad"], dg) < 1e-13
        # theta = 0.4: finite, and within the theta^(p-1) per-pair bound
        r = O.OracleFMM(x, ncrit, 0.4).evaluate(q, 6)
        assert np.all(np.isfinite(r["phi"])) and np.all(np.isfinite(r["grad"]))
        assert _rel(r["phi"], dphi) < 0.4 ** 5
        assert _rel(r["grad"], dg) < 0.4 ** 5


def test_all_coincident_is_single_leaf():
    x = np.tile(np.array([[0.25, 0.5, 0.75]]), (200, 1))
    q = W.charges(200)
    o = O.OracleFMM(x, 8, 0.4)
    assert o.num_cells == 1
    r = o.evaluate(q, 4)
    assert np.all(r["phi"] == 0) and np.all(r["grad"] == 0)


@pytest.mark.parametrize("dist,ncrit,theta,p", [("uniform", 64, 0.4, 4), ("plummer", 16, 0.35, 6)])
def test_per_leaf_evaluation_equals_full_evaluation(dist, ncrit, theta, p):
    """The per-leaf oracle (used for checks at full size) is the full evaluation."""
    x = W.positions(6000, dist)
    q = W.charges(6000)
    o = O.OracleFMM(x, ncrit, theta)
    full = o.evaluate(q, p)
    t = o.tree()
    leaves = np.nonzero(t["n_child"] == 0)[0][::3]
    idx, phi, grad = O.evaluate_leaves(o, q, p, leaves)
    assert len(set(idx.tolist())) == len(idx)
    np.testing.assert_array_equal(phi, full["phi"][idx])
    np.testing.assert_array_equal(grad, full["grad"][idx])
