"""Treecode/FMM hybrid lists on the host: identical to the oracle's, and the
argument and state checks of the hybrid entry points (no GPU needed)."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_1209_3516_amd import fmm
from paper_1209_3516_amd import workloads as W


@pytest.mark.parametrize("dist,n,ncrit,theta,leaf_first,m2p_max", [
    ("uniform", 5000, 16, 0.5, False, 8), ("plummer", 5000, 16, 0.45, False, 4),
    ("uniform", 3000, 8, 0.6, True, 3), ("uniform", 2000, 32, 0.4, False, 64)])
def test_hybrid_lists_equal_the_oracle(dist, n, ncrit, theta, leaf_first, m2p_max):
    x = W.positions(n, dist)
    o = O.OracleFMM(x, ncrit, theta, leaf_first=leaf_first, m2p_max=m2p_max)
    t = fmm.Tree(x, ncrit)
    lst = fmm.Lists(t, theta, leaf_first=leaf_first, m2p_max=m2p_max)
    for kind in (fmm.FMM_P2P, fmm.FMM_M2L, fmm.FMM_M2P):
        op, oc = o.lists(kind)
        lp, lc = lst.csr(kind)
        np.testing.assert_array_equal(op, lp)
        np.testing.assert_array_equal(oc, lc)
    s = lst.stats()
    assert s["m2p_entries"] == len(o.lists(2)[1]) > 0
    pure = fmm.Lists(t, theta, leaf_first=leaf_first)
    assert pure.stats()["m2p_entries"] == 0 and len(pure.csr(fmm.FMM_M2P)[1]) == 0
    assert s["m2l_entries"] + s["m2p_entries"] == pure.stats()["m2l_entries"]


def test_hybrid_arguments_and_unsupported_paths():
    L = fmm.lib()
    x = W.uniform_cube(3000, seed=41)
    t = fmm.Tree(x, 8)
    h = ctypes.c_void_p()
    for bad in (-1, 65):
        assert L.fmm_traverse_hybrid(t._h, 0.5, 0, bad, ctypes.byref(h)) == fmm.FMM_EINVAL
    assert L.fmm_traverse_hybrid(t._h, 1.5, 0, 4, ctypes.byref(h)) == fmm.FMM_EINVAL
    zero = fmm.Lists(t, 0.5, m2p_max=0)  # m2p_max = 0 is the pure traversal
    pure = fmm.Lists(t, 0.5)
    for kind in (fmm.FMM_P2P, fmm.FMM_M2L):
        np.testing.assert_array_equal(zero.csr(kind)[1], pure.csr(kind)[1])
    hyb = fmm.Lists(t, 0.5, m2p_max=8)
    with pytest.raises(ValueError):
        fmm.Lists(t, 0.5, m2p_max=8, device=True)
    o = fmm._EvalOpts(4, fmm.FMM_MIXED, -1, 0)
    dummy = ctypes.c_void_p(16)
    # the backward needs the symmetric operator; ranges are not implemented
    assert L.fmm_evaluate_backward(t._h, hyb._h, ctypes.byref(o), dummy, dummy, dummy, None,
                                   dummy, dummy, None) == fmm.FMM_ESTATE
    assert b"hybrid" in L.fmm_last_error()
    assert L.fmm_evaluate_range(t._h, hyb._h, ctypes.byref(o), 0, 3000, dummy, dummy, None,
                                None) == fmm.FMM_EINVAL
