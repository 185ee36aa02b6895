"""Host tests of the mutual P2P's work plan (fmm_mutual_plan_stats), no GPU.

The plan evaluates each unordered pair of P2P leaves {A, B} once, in the item
of the lower-numbered leaf, and the pairs within a leaf one-sided.  Its counts
are checked against the same counts recomputed in numpy from the P2P lists:
  * body pairs of the leaf pairs A < B, and ordered pairs within leaves; twice
    the first plus the second is the list's directed pair count;
  * partial slots of the source side: sum over leaf pairs A < B of n_B;
  * runs: one per leaf pair A < B; items: one per leaf and chunk, the chunks
    recounted with the plan's rule (8192 sources, 256 runs).
Refusals: leaves of more than 64 bodies, the 32-bit offset limit.
"""
import numpy as np
import pytest

from paper_1209_3516_amd import fmm
from paper_1209_3516_amd import workloads as W


def chunks_of_row(na, upper_sizes, has_self):
    """Chunks of one row: a chunk closes before a leaf whose bodies would take
    it past 8192 sources (its own leaf's bodies count when the chunk holds the
    self pair) or that would be its 257th leaf."""
    n_chunks, src, runs, self_ = 0, 0, 0, has_self
    for nb in upper_sizes:
        if (src + (na if self_ else 0) + nb > 8192 and (src > 0 or self_)) or runs >= 256:
            n_chunks += 1
            src, runs, self_ = 0, 0, False
        src += nb
        runs += 1
    return n_chunks + (1 if (src > 0 or self_ or n_chunks == 0) else 0)


def counts_from_lists(tree, lists):
    v = tree.view()
    ptr, col = lists.csr(fmm.FMM_P2P)
    nb = v["n_body"]
    rows = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    upper = col > rows
    self_ = col == rows
    items = 0
    for a in np.flatnonzero(v["n_child"] == 0):
        c = col[ptr[a]:ptr[a + 1]]
        items += chunks_of_row(int(nb[a]), [int(nb[b]) for b in c[c > a]], bool(np.any(c == a)))
    return dict(upper_pairs=int(np.sum(nb[rows[upper]] * nb[col[upper]])),
                self_pairs=int(np.sum(nb[rows[self_]] * (nb[rows[self_]] - 1))),
                source_slots=int(np.sum(nb[col[upper]])),
                runs=int(np.sum(upper)), items=items,
                leaves=int(np.sum(v["n_child"] == 0)))


CASES = [
    ("uniform", 20_000, 64, 0.4, 0),
    ("plummer", 20_000, 16, 0.35, 0),
    ("uniform", 3_000, 1, 0.5, 0),
    ("plummer", 6_000, 40, 0.35, 0),
    ("uniform", 8_000, 24, 0.6, 0),
    ("uniform", 10_000, 32, 0.4, 16),  # hybrid lists: the P2P list is unchanged
]


@pytest.mark.parametrize("case", CASES, ids=["-".join(map(str, c)) for c in CASES])
@pytest.mark.parametrize("leaf_first", [False, True])
def test_mutual_plan_counts(case, leaf_first):
    dist, n, ncrit, theta, m2p = case
    t = fmm.Tree(W.positions(n, dist), ncrit)
    lst = fmm.Lists(t, theta, leaf_first=leaf_first, m2p_max=m2p)
    got = lst.mutual_plan_stats()
    ref = counts_from_lists(t, lst)
    for k in ("upper_pairs", "self_pairs", "source_slots", "runs", "items"):
        assert got[k] == ref[k], k
    assert 2 * got["upper_pairs"] + got["self_pairs"] == lst.stats()["p2p_pairs"]
    assert got["items"] >= ref["leaves"]


def test_mutual_plan_chunks_long_rows():
    """Rows of more than 8192 upper sources or 256 upper leaves take several
    items; every pair is still counted once."""
    t = fmm.Tree(W.uniform_cube(20_000, seed=31), 64)
    lst = fmm.Lists(t, 0.15)
    got = lst.mutual_plan_stats()
    ref = counts_from_lists(t, lst)
    assert got["items"] == ref["items"] > ref["leaves"]
    assert got["upper_pairs"] == ref["upper_pairs"] and got["runs"] == ref["runs"]
    assert 2 * got["upper_pairs"] + got["self_pairs"] == lst.stats()["p2p_pairs"]


def test_mutual_plan_refuses_large_leaves():
    t = fmm.Tree(W.uniform_cube(4000), 200)
    lst = fmm.Lists(t, 0.4)
    with pytest.raises(fmm.FMMError) as e:
        lst.mutual_plan_stats()
    assert e.value.code == fmm.FMM_EINVAL
    assert b"at most 64 bodies" in fmm.lib().fmm_last_error()


def test_mutual_plan_refuses_past_the_offset_limit(monkeypatch):
    t = fmm.Tree(W.uniform_cube(5000), 32)
    lst = fmm.Lists(t, 0.4)
    need = lst.mutual_plan_stats()["source_slots"]
    monkeypatch.setenv("FMM_PLAN_LIMIT", str(need - 1))
    with pytest.raises(fmm.FMMError) as e:
        lst.mutual_plan_stats()
    assert e.value.code == fmm.FMM_EINVAL
    assert b"too large" in fmm.lib().fmm_last_error()
    monkeypatch.setenv("FMM_PLAN_LIMIT", str(need))
    assert lst.mutual_plan_stats()["source_slots"] == need
