"""Pins of the oracle's M2P operator and of the treecode/FMM hybrid lists
(M2P for accepted pairs whose target is a small leaf), against facts that do
not come from the M2P code itself:

* a single body is its own multipole: M2P is exact for every p;
* the multipole series of a cluster converges like (a/R)^p (the theta^p
  bound of section 3.2) and its error falls with p;
* at the target centre, M2P's potential is L2P(M2L(M)) (the local
  expansion's constant term), and its gradient is that of L2P(M2L) one order
  higher with the multipole padded by zeros;
* the hybrid lists are the pure lists with the accepted pairs split: M2L and
  M2P together are the pure M2L list, P2P is unchanged, every M2P target is a
  leaf of at most m2p_max bodies, every ordered body pair is covered once;
* the hybrid evaluation is no less accurate than the pure FMM against the
  direct sum, and tends to it as theta -> 0.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1209_3516_amd import workloads as W

M2P = 2


def _cluster(n, a, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d *= (a * rng.random(n) ** (1 / 3) / np.linalg.norm(d, axis=1))[:, None]
    return d, rng.uniform(-1, 1, n)


def _direct(x, q, y):
    d = x[None, :, :] - y[:, None, :]
    r = np.linalg.norm(d, axis=2)
    phi = (q / r).sum(1)
    grad = (q[None, :, None] * d / r[:, :, None] ** 3).sum(1)
    return phi, grad


@pytest.mark.parametrize("p", range(1, 9))
def test_m2p_single_body_is_exact(p):
    xj = np.array([[0.3, -0.2, 0.7]])
    M = O.p2m(p, xj[0], xj, np.array([1.7]))
    y = np.array([[2.0, 1.0, -1.0], [-0.4, 0.9, 3.0]])
    phi, grad = O.m2p(p, xj[0], M, y)
    ref_phi, ref_grad = _direct(xj, np.array([1.7]), y)
    np.testing.assert_allclose(phi, ref_phi, rtol=1e-14)
    np.testing.assert_allclose(grad, ref_grad, rtol=1e-13)


@pytest.mark.parametrize("R", [3.0, 5.0])
def test_m2p_converges_like_a_over_r_to_the_p(R):
    a = 1.0
    X = np.array([0.1, 0.2, -0.3])
    d, q = _cluster(40, a, seed=5)
    x = X + d
    rng = np.random.default_rng(6)
    u = rng.normal(size=(20, 3))
    y = X + R * u / np.linalg.norm(u, axis=1)[:, None]
    ref_phi, ref_grad = _direct(x, q, y)
    err_phi, err_grad = [], []
    for p in range(1, 9):
        phi, grad = O.m2p(p, X, O.p2m(p, X, x, q), y)
        e = np.abs(phi - ref_phi).max()
        bound = np.abs(q).sum() * (a / R) ** p / (R - a)
        assert e <= bound * (1 + 1e-12) + 1e-15, (p, e, bound)
        err_phi.append(e)
        err_grad.append(np.abs(grad - ref_grad).max())
    assert all(b < a_ for a_, b in zip(err_phi, err_phi[1:]))
    assert all(b < a_ for a_, b in zip(err_grad[1:], err_grad[2:]))
    assert err_grad[-1] < 1e-3 * err_grad[0]


@pytest.mark.parametrize("p", [2, 4, 6])
def test_m2p_at_target_centre_matches_m2l_then_l2p(p):
    rng = np.random.default_rng(7 + p)
    XB = np.array([0.0, 0.0, 0.0])
    XA = np.array([2.5, -1.0, 1.5])
    M = rng.normal(size=O.num_terms(p))
    phi, grad = O.m2p(p, XB, M, XA[None, :])
    lphi, _ = O.l2p(p, XA, O.m2l(p, XA, XB, M), XA[None, :])
    np.testing.assert_allclose(phi, lphi, rtol=1e-13)
    # one order higher, the multipole padded with zero terms of degree p
    # (terms are ordered by degree, so the padding goes at the end)
    M1 = np.concatenate([M, np.zeros(O.num_terms(p + 1) - O.num_terms(p))])
    _, lgrad = O.l2p(p + 1, XA, O.m2l(p + 1, XA, XB, M1), XA[None, :])
    np.testing.assert_allclose(grad, lgrad, rtol=1e-12, atol=1e-15 * np.abs(lgrad).max())


def _pairs(o, kind):
    ptr, col = o.lists(kind)
    rows = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    return set(zip(rows.tolist(), col.tolist())), rows, col


@pytest.mark.parametrize("dist,n,ncrit,theta,leaf_first,m2p_max", [
    ("uniform", 1500, 8, 0.5, False, 4), ("plummer", 1500, 16, 0.6, False, 8),
    ("uniform", 1200, 4, 0.4, True, 3), ("uniform", 800, 8, 0.5, False, 1000)])
def test_hybrid_lists_split_the_accepted_pairs(dist, n, ncrit, theta, leaf_first, m2p_max):
    x = W.positions(n, dist)
    pure = O.OracleFMM(x, ncrit, theta, leaf_first=leaf_first)
    hyb = O.OracleFMM(x, ncrit, theta, leaf_first=leaf_first, m2p_max=m2p_max)
    t = hyb.tree()
    p2p_pure, _, _ = _pairs(pure, O.P2P)
    m2l_pure, _, _ = _pairs(pure, O.M2L)
    p2p, _, _ = _pairs(hyb, O.P2P)
    m2l, mrows, _ = _pairs(hyb, O.M2L)
    m2p, prows, pcol = _pairs(hyb, M2P)
    assert p2p == p2p_pure
    assert m2l | m2p == m2l_pure and not (m2l & m2p)
    assert len(m2p) > 0
    leaf_small = (t["n_child"] == 0) & (t["n_body"] <= m2p_max)
    assert np.all(leaf_small[prows])
    assert not np.any(leaf_small[mrows])
    # every ordered body pair is covered exactly once
    cover = np.zeros((n, n), np.int32)
    for a, b in p2p | m2l | m2p:
        ia = slice(t["body_begin"][a], t["body_begin"][a] + t["n_body"][a])
        ib = slice(t["body_begin"][b], t["body_begin"][b] + t["n_body"][b])
        cover[ia, ib] += 1
    assert np.all(cover == 1)
    # m2p_max = 0 is the pure FMM
    zero = O.OracleFMM(x, ncrit, theta, leaf_first=leaf_first, m2p_max=0)
    assert _pairs(zero, M2P)[0] == set() and _pairs(zero, O.M2L)[0] == m2l_pure


@pytest.mark.parametrize("p", [3, 5])
def test_hybrid_is_at_least_as_accurate_and_exact_as_theta_vanishes(p):
    n = 2000
    x = W.uniform_cube(n, seed=31)
    q = W.charges(n, seed=32)
    tg = np.arange(0, n, 7)
    ref = O.direct(x, q, tg)
    pure = O.OracleFMM(x, 8, 0.5).evaluate(q, p)
    hyb = O.OracleFMM(x, 8, 0.5, m2p_max=8).evaluate(q, p)

    def err(r):
        return (np.linalg.norm(r["phi"][tg] - ref[0]) / np.linalg.norm(ref[0]),
                np.linalg.norm(r["grad"][tg] - ref[1]) / np.linalg.norm(ref[1]))

    ep, eh = err(pure), err(hyb)
    assert eh[0] <= ep[0] * 1.05 and eh[1] <= ep[1] * 1.05, (ep, eh)
    tiny = O.OracleFMM(x, 8, 1e-3, m2p_max=8).evaluate(q, p)
    np.testing.assert_allclose(tiny["phi"][tg], ref[0], rtol=1e-12)
