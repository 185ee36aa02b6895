"""GPU dispatch orders of a full evaluation (fmm_dispatch_order), read back
from the device and checked against their definitions:

* both orders: entry 8 j + x is the j-th unit of XCD range x or -1 past its
  end; every unit (P2P work item, M2L cell) occurs once; the eight ranges
  are contiguous runs of units, in order;
* M2L, recomputed here from the lists: range x holds the cells whose work
  midpoints fall in the x-th eighth of the total work (a row costs
  ceil(length / 64) + 1), and a range's rows go by decreasing length, ties
  by cell;
* host-built lists (ordered at their upload) and device-built lists give
  the same orders.
Whether the orders leave results unchanged is checked elsewhere: the target
range evaluations, which take no order, reassemble the full evaluation bit
for bit (tests/test_gpu_traverse.py).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1209_3516_amd import fmm  # noqa: E402
from paper_1209_3516_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def expected_m2l_ranges(ptr):
    ln = np.diff(ptr)
    c = (ln + 63) // 64 + 1
    pre = np.concatenate([[0], np.cumsum(c)[:-1]])
    tot = int(c.sum())
    return np.minimum(7, (8 * (2 * pre + c)) // (2 * tot)), ln


def check_ranges(order, n_units):
    """The common structure; returns the units of each range."""
    assert order.size % 8 == 0
    valid = order[order >= 0]
    assert np.array_equal(np.sort(valid), np.arange(n_units))
    ranges, widest, last = [], 0, -1
    for x in range(8):
        col = order[x::8]
        k = int(np.sum(col >= 0))
        widest = max(widest, k)
        assert np.all(col[:k] >= 0) and np.all(col[k:] == -1)
        units = np.sort(col[:k])
        if k:
            assert units[-1] - units[0] == k - 1  # contiguous
            assert units[0] == last + 1           # ranges in order
            last = units[-1]
        ranges.append(col[:k])
    assert order.size == 8 * widest
    return ranges


def check_orders(t, lst):
    po = lst.dispatch_order(fmm.FMM_P2P)
    check_ranges(po, lst.stats()["p2p_work_items"])

    ptr, _ = lst.csr(fmm.FMM_M2L)
    mo = lst.dispatch_order(fmm.FMM_M2L)
    ranges = check_ranges(mo, ptr.size - 1)
    xr, ln = expected_m2l_ranges(ptr)
    for x, cells in enumerate(ranges):
        # exactly the cells the rule assigns to range x
        assert np.array_equal(np.sort(cells), np.flatnonzero(xr == x))
        # by decreasing length, ties by cell index
        assert np.array_equal(np.lexsort((cells, -ln[cells])), np.arange(cells.size))
    return po, mo


CASES = [
    ("uniform", 50_000, 32, 0.4),
    ("plummer", 50_000, 16, 0.35),
    ("uniform", 3_000, 1, 0.5),
    ("uniform", 5, 64, 0.5),  # one cell: a single M2L row of length 0, one work item
]


@pytest.mark.parametrize("case", CASES, ids=["-".join(map(str, c)) for c in CASES])
def test_dispatch_orders(case):
    dist, n, ncrit, theta = case
    print("case", case, flush=True)
    x = W.positions(n, dist)
    q = torch.tensor(W.charges(n, seed=7), dtype=torch.float32, device="cuda:0")
    t = fmm.Tree(x, ncrit)
    host = fmm.Lists(t, theta)
    with pytest.raises(fmm.FMMError) as e:
        host.dispatch_order(fmm.FMM_P2P)  # not on the device before the first evaluation
    assert e.value.code == fmm.FMM_ESTATE
    fmm.evaluate(t, host, q, 4)
    torch.cuda.synchronize()
    po_h, mo_h = check_orders(t, host)
    dev = fmm.Lists(t, theta, device=True)
    po_d, mo_d = check_orders(t, dev)
    assert np.array_equal(po_h, po_d) and np.array_equal(mo_h, mo_d)


def test_dispatch_order_buffer_too_small():
    import ctypes
    t = fmm.Tree(W.uniform_cube(4000, seed=8), 16)
    lst = fmm.Lists(t, 0.4, device=True)
    n = ctypes.c_int64()
    L = fmm.lib()
    assert L.fmm_dispatch_order(lst._h, fmm.FMM_M2L, None, 0, ctypes.byref(n)) == fmm.FMM_OK
    assert n.value > 0
    buf = (ctypes.c_int32 * n.value)()
    assert L.fmm_dispatch_order(lst._h, fmm.FMM_M2L, buf, n.value - 1,
                                ctypes.byref(n)) == fmm.FMM_EINVAL
    assert L.fmm_dispatch_order(lst._h, fmm.FMM_M2L, buf, n.value,
                                ctypes.byref(n)) == fmm.FMM_OK
