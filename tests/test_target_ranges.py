"""Target ranges (one GPU's share of the targets) on the host: the weighted
Morton partition and the argument checks of fmm_evaluate_range."""
import ctypes

import numpy as np
import pytest

from paper_1209_3516_amd import fmm
from paper_1209_3516_amd import workloads as W


def _leaf_weights(tree, lists, w_m2l):
    """Per-leaf work as documented (P2P pairs + w_m2l * M2L entries shared down
    by bodies), recomputed here from the views, in Morton order."""
    v = tree.view()
    nb, par, nch, bb = v["n_body"], v["parent"], v["n_child"], v["body_begin"]
    pp, pc = lists.csr(fmm.FMM_P2P)
    mp, _ = lists.csr(fmm.FMM_M2L)
    share = np.zeros(len(nb))
    for c in range(len(nb)):  # parents precede children
        share[c] = (share[par[c]] if par[c] >= 0 else 0.0) + (mp[c + 1] - mp[c]) / nb[c]
    out = []
    for c in np.flatnonzero(nch == 0):
        src = pc[pp[c]:pp[c + 1]]
        pairs = float(sum(nb[c] * (nb[b] - (1 if b == c else 0)) for b in src))
        out.append((bb[c], pairs + w_m2l * share[c] * nb[c]))
    out.sort()
    return np.array([s for s, _ in out]), np.array([w for _, w in out])


@pytest.mark.parametrize("kind,n,ncrit,G", [("uniform", 20_000, 32, 8), ("plummer", 20_000, 16, 5),
                                            ("uniform", 3_000, 64, 1), ("uniform", 300, 64, 40)])
def test_partition_is_contiguous_leaf_aligned_and_balanced(kind, n, ncrit, G):
    x = W.uniform_cube(n, seed=110) if kind == "uniform" else W.plummer(n, seed=110)
    t = fmm.Tree(x, ncrit)
    lst = fmm.Lists(t, 0.5)
    w = fmm.m2l_weight(4)
    bounds = fmm.partition(t, lst, G, p=4)
    starts, weights = _leaf_weights(t, lst, w)
    assert bounds[0] == 0 and bounds[-1] == n and len(bounds) == G + 1
    assert np.all(np.diff(bounds) >= 0)
    for b in bounds[1:-1]:
        assert b in set(starts.tolist()) or b == n
    # each range's weight is within one leaf of the ideal share
    part = np.searchsorted(bounds, starts, side="right") - 1
    per = np.bincount(part, weights=weights, minlength=G)
    assert per.sum() == pytest.approx(weights.sum())
    assert np.all(np.abs(per - weights.sum() / G) <= weights.max() + 1e-9 * weights.sum())


def test_range_arguments_are_checked_without_gpu():
    L = fmm.lib()
    x = W.uniform_cube(2000, seed=111)
    t = fmm.Tree(x, 16)
    lst = fmm.Lists(t, 0.5)
    v = t.view()
    leaf_starts = np.sort(v["body_begin"][v["n_child"] == 0])
    inner = int(leaf_starts[1]) + 1  # inside a leaf of more than one body
    assert inner not in set(leaf_starts.tolist())
    o = fmm._EvalOpts(4, fmm.FMM_MIXED, -1, 0)
    dummy = ctypes.c_void_p(16)
    for b0, b1 in ((-1, 10), (5, 4), (0, 2001), (inner, 2000), (0, inner)):
        rc = L.fmm_evaluate_range(t._h, lst._h, ctypes.byref(o), b0, b1, dummy, dummy, None, None)
        assert rc == fmm.FMM_EINVAL, (b0, b1)
    # an empty range is a no-op, even without a GPU
    assert L.fmm_evaluate_range(t._h, lst._h, ctypes.byref(o), 7, 7, dummy, dummy, None,
                                None) == fmm.FMM_OK
    bounds = (ctypes.c_int64 * 3)()
    assert L.fmm_partition_targets(t._h, lst._h, 0, 1.0, bounds) == fmm.FMM_EINVAL
    assert L.fmm_partition_targets(t._h, lst._h, 2, -1.0, bounds) == fmm.FMM_EINVAL
    other = fmm.Tree(x, 16)
    assert L.fmm_partition_targets(other._h, lst._h, 2, 1.0, bounds) == fmm.FMM_ESTATE
