"""Pins of the oracle's box-centred cell geometry (cell centres at the centres
of the Morton cubes; the geometric centre of the paper's Table 3).

* geometry: every body of a cell lies in the cube of side 2h / 2^L about the
  cell's centre; a child's centre is its parent's centre moved by a quarter
  of the parent's side along each axis (towards the child's octant, read from
  the Morton key); the radius is the largest centre-to-body distance;
* lists (brute force): every ordered body pair is covered exactly once, every
  M2L entry meets the MAC, P2P entries are leaf pairs that fail it, the lists
  are symmetric;
* the translation vector of every M2L entry between cells of one level is an
  integer multiple of the level's cube side, so the vectors repeat;
* the evaluation against the O(N^2) direct sum: small error that falls with p.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1209_3516_amd import workloads as W

CASES = [("uniform", 1500, 16, 0.4), ("plummer", 1500, 8, 0.35), ("uniform", 1200, 1, 0.5)]


def _side(x, level):
    lo, hi = x.min(0), x.max(0)
    h = 0.5 * (hi - lo).max()
    return 2.0 * h / 2.0 ** level


@pytest.mark.parametrize("dist,n,ncrit,theta", CASES)
def test_box_tree_geometry(dist, n, ncrit, theta):
    x = W.positions(n, dist)
    o = O.OracleFMM(x, ncrit, theta, box_centres=True)
    t = o.tree()
    xs = x[t["perm"]]
    tol = 1e-12 * np.abs(x).max()
    for c in range(o.num_cells):
        b0, nb, lev = t["body_begin"][c], t["n_body"][c], int(t["level"][c])
        w = _side(x, lev)
        pts = xs[b0:b0 + nb]
        assert np.all(np.abs(pts - t["center"][c]) <= 0.5 * w + tol)
        dist_c = np.sqrt(((pts - t["center"][c]) ** 2).sum(1))
        assert t["radius"][c] >= dist_c.max() * (1 - 1e-15)
        assert t["radius"][c] <= dist_c.max() * (1 + 1e-15)
        for k in range(t["n_child"][c]):
            ch = t["child_begin"][c] + k
            octant = int((int(t["keys"][t["body_begin"][ch]]) >> (3 * (20 - lev))) & 7)
            for d in range(3):
                sign = 1.0 if (octant >> d) & 1 else -1.0
                want = t["center"][c][d] + sign * 0.25 * w
                assert abs(t["center"][ch][d] - want) <= tol


@pytest.mark.parametrize("leaf_first", [False, True])
@pytest.mark.parametrize("dist,n,ncrit,theta", CASES)
def test_box_lists_partition_mac_symmetry(dist, n, ncrit, theta, leaf_first):
    x = W.positions(n, dist)
    o = O.OracleFMM(x, ncrit, theta, leaf_first=leaf_first, box_centres=True)
    t = o.tree()
    cover = np.zeros((n, n), dtype=np.int32)
    is_leaf = t["n_child"] == 0
    for kind in (O.P2P, O.M2L):
        ptr, col = o.lists(kind)
        rows = np.repeat(np.arange(o.num_cells), np.diff(ptr))
        pairs = set(zip(rows.tolist(), col.tolist()))
        assert pairs == {(b, a) for a, b in pairs}
        d = t["center"][rows] - t["center"][col]
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        s = t["radius"][rows] + t["radius"][col]
        mac = (theta * theta) * d2 > s * s
        if kind == O.M2L:
            assert np.all(mac)
        else:
            assert np.all(is_leaf[rows]) and np.all(is_leaf[col])
            if not leaf_first:
                assert not np.any(mac)
        for a, b in zip(rows, col):
            ia = slice(t["body_begin"][a], t["body_begin"][a] + t["n_body"][a])
            ib = slice(t["body_begin"][b], t["body_begin"][b] + t["n_body"][b])
            cover[ia, ib] += 1
    assert np.all(cover == 1)


def test_box_translations_are_lattice_vectors_and_repeat():
    """X_A - X_B is an integer multiple of half the side of the finer of the
    two cells' cubes (a whole multiple of the side when both are on one
    level), and few distinct (level A, level B, vector) triples serve all
    entries."""
    x = W.uniform_cube(20000)
    o = O.OracleFMM(x, 32, 0.4, box_centres=True)
    t = o.tree()
    ptr, col = o.lists(O.M2L)
    rows = np.repeat(np.arange(o.num_cells), np.diff(ptr))
    la, lb = t["level"][rows], t["level"][col]
    fine = np.maximum(la, lb)
    w = np.array([_side(x, L) for L in range(22)])[fine]
    r = (t["center"][rows] - t["center"][col]) / (0.5 * w[:, None])
    assert np.all(np.abs(r - np.round(r)) < 1e-9)
    r = np.round(r).astype(np.int64)
    same = la == lb
    assert np.all(r[same] % 2 == 0)
    key = np.concatenate([la[:, None], lb[:, None], r], axis=1)
    distinct = np.unique(key, axis=0).shape[0]
    assert same.mean() > 0.5
    assert distinct * 20 < len(col)  # each vector serves many entries


def test_box_lists_differ_from_bounding_box_centres():
    x = W.uniform_cube(5000, seed=9)
    a = O.OracleFMM(x, 16, 0.4)
    b = O.OracleFMM(x, 16, 0.4, box_centres=True)
    assert not np.array_equal(a.tree()["center"], b.tree()["center"])
    assert not np.array_equal(a.lists(O.M2L)[1], b.lists(O.M2L)[1])


def test_box_evaluation_against_direct_sum():
    n = 2000
    x = W.positions(n, "plummer")
    q = W.charges(n)
    o = O.OracleFMM(x, 16, 0.5, box_centres=True)
    dphi, dg = O.direct(x, q)
    errs = []
    for p in (2, 4, 6, 8):
        r = o.evaluate(q, p)
        errs.append(np.linalg.norm(r["grad"] - dg) / np.linalg.norm(dg))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-4
