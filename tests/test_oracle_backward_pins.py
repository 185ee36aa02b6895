"""Pins of the oracle's dipole-source and Hessian machinery, and of the adjoint
used for a loss that also depends on the gradient output:

  L = sum_i w_i phi_i + sum_i v_i . grad_i
  dL/dq   = Phi            (potential of charges w plus dipoles -v)
  dL/dx   = w * grad[q] + q * grad Phi + H[q] v

With the tree, lists, centres and radii frozen, the method is an exactly
differentiable function, so finite differences of the oracle's own forward
evaluation check these formulas (and every piece they use).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1209_3516_amd import workloads as W


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.mark.parametrize("p", [3, 5, 8])
def test_single_dipole_is_exact(p):
    XB = np.array([0.2, -0.1, 0.4])
    XA = np.array([1.3, 0.6, -0.5])
    s = np.array([0.3, -0.7, 0.5])
    M = O.p2m_dipole(p, XB, XB[None, :], s[None, :])
    ex = [tuple(e) for e in O.term_exponents(p)]
    want_M = np.zeros(len(ex))
    for a, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        want_M[ex.index(e)] = s[a]
    np.testing.assert_allclose(M, want_M, atol=1e-15)
    L = O.m2l(p, XA, XB, M)
    f, g = O.l2p(p, XA, L, XA[None, :])
    d = XB - XA
    r = np.linalg.norm(d)
    assert f[0] == pytest.approx(s @ d / r ** 3, rel=1e-14)
    np.testing.assert_allclose(g[0], -s / r ** 3 + 3 * (s @ d) * d / r ** 5, rtol=1e-13)


def test_dipole_is_limit_of_two_charges():
    rng = np.random.default_rng(50)
    src = rng.uniform(0, 1, (20, 3))
    s = rng.standard_normal((20, 3))
    tgt = rng.uniform(2, 3, (5, 3))
    xyz = np.concatenate([tgt, src])
    q0 = np.zeros(25)
    s_all = np.concatenate([np.zeros((5, 3)), s])
    f, g, _ = O.direct_general(xyz, q0, s_all, targets=np.arange(5))
    h = 1e-4
    plus, minus = src - 0.5 * h * s, src + 0.5 * h * s  # +1/h at x - hs/2, -1/h at x + hs/2
    xyz2 = np.concatenate([tgt, plus, minus])
    q2 = np.concatenate([np.zeros(5), np.full(20, 1 / h), np.full(20, -1 / h)])
    f2, g2 = O.direct(xyz2, q2, np.arange(5))
    assert rel(f, f2) < 1e-7
    assert rel(g, g2) < 1e-7


def test_direct_hessian_matches_finite_differences():
    rng = np.random.default_rng(51)
    xyz = rng.uniform(0, 1, (60, 3))
    q = rng.uniform(-1, 1, 60)
    tg = np.arange(10)
    v = rng.standard_normal((10, 3))
    _, _, hv = O.direct_general(xyz, q, None, tg, v)
    h = 1e-5
    for k in range(10):
        xp, xm = xyz.copy(), xyz.copy()
        xp[k] += h * v[k]
        xm[k] -= h * v[k]
        gp = O.direct(xp, q, [k])[1][0]
        gm = O.direct(xm, q, [k])[1][0]
        np.testing.assert_allclose(hv[k], (gp - gm) / (2 * h), rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("p", [2, 4, 7])
def test_l2p_hessian_is_derivative_of_l2p_gradient(p):
    rng = np.random.default_rng(52)
    L = rng.standard_normal(O.num_terms(p))
    XA = rng.uniform(0, 1, 3)
    y = XA + rng.uniform(-0.2, 0.2, (6, 3))
    v = rng.standard_normal((6, 3))
    hv = O.l2p_hessian(p, XA, L, y, v)
    h = 1e-6
    _, gp = O.l2p(p, XA, L, y + h * v)
    _, gm = O.l2p(p, XA, L, y - h * v)
    np.testing.assert_allclose(hv, (gp - gm) / (2 * h), rtol=1e-6, atol=1e-6)


def test_general_fmm_tiny_theta_is_direct_sum():
    n = 500
    x = W.uniform_cube(n, seed=53)
    q = W.charges(n, seed=54)
    s = W.dipoles(n, seed=55)
    v = W.dipoles(n, seed=56)
    o = O.OracleFMM(x, 4, 1e-6)
    f, g, _ = O.evaluate_general(o, 4, q, s=s)
    df, dg, _ = O.direct_general(x, q, s)
    assert rel(f, df) < 1e-13 and rel(g, dg) < 1e-13
    _, _, hv = O.evaluate_general(o, 4, q, v=v)
    _, _, dhv = O.direct_general(x, q, None, None, v)
    assert rel(hv, dhv) < 1e-13


def test_general_fmm_error_falls_with_p():
    n = 3000
    x = W.uniform_cube(n, seed=57)
    q = W.charges(n, seed=58)
    s = W.dipoles(n, seed=59)
    v = W.dipoles(n, seed=60)
    o = O.OracleFMM(x, 16, 0.45)
    df, dg, _ = O.direct_general(x, q, s)
    _, _, dhv = O.direct_general(x, q, None, None, v)
    errs = []
    for p in (3, 5, 7):
        f, g, _ = O.evaluate_general(o, p, q, s=s)
        _, _, hv = O.evaluate_general(o, p, q, v=v)
        errs.append((rel(f, df), rel(g, dg), rel(hv, dhv)))
    for k in range(3):
        assert errs[2][k] < errs[1][k] < errs[0][k]


def test_adjoint_formulas_match_finite_differences():
    n = 400
    x = W.uniform_cube(n, seed=61)
    q = W.charges(n, seed=62)
    w = W.weights(n, seed=63)
    v = W.dipoles(n, seed=64)
    p = 4
    o = O.OracleFMM(x, 16, 0.5)

    def loss(xx, qq):
        O.set_positions(o, xx)
        r = o.evaluate(qq, p)
        return float(w @ r["phi"] + np.sum(v * r["grad"]))

    O.set_positions(o, x)
    _, gq, hv = O.evaluate_general(o, p, q, v=v)
    Phi, gPhi, _ = O.evaluate_general(o, p, w, s=-v)
    dq = Phi
    dx = w[:, None] * gq + q[:, None] * gPhi + hv
    rng = np.random.default_rng(65)
    h = 1e-6
    for _ in range(12):
        j = int(rng.integers(n))
        qp, qm = q.copy(), q.copy()
        qp[j] += h
        qm[j] -= h
        fd = (loss(x, qp) - loss(x, qm)) / (2 * h)
        assert abs(fd - dq[j]) <= 1e-6 * max(1.0, abs(dq[j]))
    for _ in range(12):
        i, d = int(rng.integers(n)), int(rng.integers(3))
        xp, xm = x.copy(), x.copy()
        xp[i, d] += h
        xm[i, d] -= h
        fd = (loss(xp, q) - loss(xm, q)) / (2 * h)
        scale = max(1.0, abs(dx[i, d]), math.sqrt(np.mean(dx ** 2)))
        assert abs(fd - dx[i, d]) <= 1e-5 * scale, (i, d, fd, dx[i, d])
    O.set_positions(o, x)
