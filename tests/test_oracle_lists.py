"""Invariants of the oracle's tree and dual-tree-traversal lists.

* tree: children partition their parent's bodies; leaves hold <= ncrit bodies
  (unless at the depth cap); breadth-first numbering; octant geometry of the
  Morton order; expansion centre = midpoint of the tight bounding box and
  radius = largest centre-to-body distance (rectangular cells, section 3.3);
* lists: every ordered body pair (i, j) is covered by exactly one list entry
  (brute force); every M2L entry meets the MAC (section 3.2); in MAC-first mode
  every P2P entry is leaf x leaf and fails it; the lists are symmetric;
  rows are sorted.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1209_3516_amd import workloads as W


def _mac(t, a, b, theta):
    d = t["center"][a] - t["center"][b]
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    s = t["radius"][a] + t["radius"][b]
    return (theta * theta) * d2 > s * s


def _rows(ptr):
    return np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))


CASES = [("uniform", 1500, 16, 0.4), ("uniform", 1500, 1, 0.5), ("plummer", 1500, 8, 0.35),
         ("uniform", 800, 64, 0.2), ("plummer", 1200, 32, 0.6)]


@pytest.mark.parametrize("dist,n,ncrit,theta", CASES)
def test_tree_invariants(dist, n, ncrit, theta):
    x = W.positions(n, dist)
    o = O.OracleFMM(x, ncrit, theta)
    t = o.tree()
    nc = o.num_cells
    assert sorted(t["perm"].tolist()) == list(range(n))
    assert np.all(np.diff(t["keys"].astype(np.float64)) >= 0)
    assert np.all(np.diff(t["level"]) >= 0)  # breadth first
    xs = x[t["perm"]]
    for c in range(nc):
        b0, nb = t["body_begin"][c], t["n_body"][c]
        if t["n_child"][c] == 0:
            assert nb <= ncrit or t["level"][c] == 21
        else:
            assert nb > ncrit
            ch = np.arange(t["child_begin"][c], t["child_begin"][c] + t["n_child"][c])
            assert np.all(t["parent"][ch] == c)
            assert np.all(t["level"][ch] == t["level"][c] + 1)
            assert t["body_begin"][ch[0]] == b0
            assert np.all(t["body_begin"][ch[1:]] == t["body_begin"][ch[:-1]] + t["n_body"][ch[:-1]])
            assert t["n_body"][ch].sum() == nb
        pts = xs[b0:b0 + nb]
        lo, hi = pts.min(0), pts.max(0)
        np.testing.assert_array_equal(t["center"][c], 0.5 * (lo + hi))
        dist_c = np.sqrt(((pts - t["center"][c]) ** 2).sum(1))
        assert t["radius"][c] >= dist_c.max() * (1 - 1e-15)
        assert t["radius"][c] <= dist_c.max() * (1 + 1e-15)


def test_morton_octant_geometry():
    x = W.uniform_cube(4000, seed=5)
    o = O.OracleFMM(x, 8, 0.4)
    t = o.tree()
    lo, hi = x.min(0), x.max(0)
    c = 0.5 * (lo + hi)
    xs = x[t["perm"]]
    ch = np.arange(t["child_begin"][0], t["child_begin"][0] + t["n_child"][0])
    assert len(ch) == 8
    for octant, cell in enumerate(ch):
        pts = xs[t["body_begin"][cell]:t["body_begin"][cell] + t["n_body"][cell]]
        for d in range(3):  # x is the lowest bit of an octant number, z the highest
            if (octant >> d) & 1:
                assert np.all(pts[:, d] >= c[d])
            else:
                assert np.all(pts[:, d] < c[d])


@pytest.mark.parametrize("leaf_first", [False, True])
@pytest.mark.parametrize("dist,n,ncrit,theta", CASES)
def test_lists_partition_mac_symmetry(dist, n, ncrit, theta, leaf_first):
    x = W.positions(n, dist)
    o = O.OracleFMM(x, ncrit, theta, leaf_first=leaf_first)
    t = o.tree()
    cover = np.zeros((n, n), dtype=np.int32)
    is_leaf = t["n_child"] == 0
    for kind in (O.P2P, O.M2L):
        ptr, col = o.lists(kind)
        rows = _rows(ptr)
        for r in range(o.num_cells):  # sources ascend within a row
            assert np.all(np.diff(col[ptr[r]:ptr[r + 1]]) > 0)
        pairs = set(zip(rows.tolist(), col.tolist()))
        assert pairs == {(b, a) for a, b in pairs}  # symmetric
        mac = _mac(t, rows, col, theta)
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


def test_lists_single_leaf_and_empty():
    x = W.uniform_cube(10)
    o = O.OracleFMM(x, 64, 0.4)
    ptr, col = o.lists(O.P2P)
    assert o.num_cells == 1 and list(ptr) == [0, 1] and list(col) == [0]
    o = O.OracleFMM(np.zeros((0, 3)), 64, 0.4)
    assert o.num_cells == 0
    assert list(o.lists(O.P2P)[0]) == [0]


def test_leaf_first_has_more_p2p():
    x = W.uniform_cube(5000, seed=9)
    a = O.OracleFMM(x, 16, 0.4, leaf_first=False)
    b = O.OracleFMM(x, 16, 0.4, leaf_first=True)
    assert len(b.lists(O.P2P)[1]) > len(a.lists(O.P2P)[1])


@pytest.mark.parametrize("dist,leaf_first", [("plummer", False), ("uniform", True),
                                             ("uniform", False)])
def test_restricted_traversal_keeps_the_rows_of_the_chosen_paths(dist, leaf_first):
    """The restricted traversal (used for per-leaf checks at sizes where the
    whole lists are large) gives, for every chosen leaf and each of its
    ancestors, the whole traversal's row, and no other rows; the per-leaf
    evaluation on it is identical."""
    x = W.positions(20_000, dist)
    q = W.charges(20_000)
    full = O.OracleFMM(x, 16, 0.4, leaf_first=leaf_first)
    t = full.tree()
    leaves = np.nonzero(t["n_child"] == 0)[0]
    pick = np.sort(np.random.default_rng(5).choice(leaves, 25, replace=False)).astype(np.int32)
    part = O.OracleFMM(x, 16, 0.4, leaf_first=leaf_first, select_leaves=lambda tt: pick)
    on_path = np.zeros(full.num_cells, bool)
    for c in pick:
        while c >= 0:
            on_path[c] = True
            c = t["parent"][c]
    for kind in (O.P2P, O.M2L):
        fp, fc = full.lists(kind)
        rp, rc = part.lists(kind)
        for c in range(full.num_cells):
            want = fc[fp[c]:fp[c + 1]] if on_path[c] else fc[:0]
            np.testing.assert_array_equal(rc[rp[c]:rp[c + 1]], want)
    a = O.evaluate_leaves(full, q, 5, pick)
    b = O.evaluate_leaves(part, q, 5, pick)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    with pytest.raises(ValueError):
        part.evaluate(q, 5)
