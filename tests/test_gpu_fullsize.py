"""Parity at full benchmark sizes, in the launch configuration bench.py times
(mixed precision, near field overlapped with the far field).

* uniform N = 10^6, p = 4: the whole oracle evaluation (all bodies) and the FP64
  direct sum on 1000 sampled targets;
* Plummer N = 10^6, p = 6, theta = 0.35, ncrit = 32: the oracle's per-leaf
  evaluation (identical arithmetic to its full evaluation) on sampled leaves,
  including the leaves with the longest P2P rows and the deepest leaves;
* uniform N = 10^7, p = 8, theta = 0.3: the FP64 direct sum on 1000 sampled
  targets (a property that holds at any size: the error is within the
  theta^p bound of an accepted pair, and no worse than at small N).
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1209_3516_amd import fmm  # noqa: E402
from paper_1209_3516_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def run_gpu(x, q, cfg, precision="mixed"):
    t0 = time.perf_counter()
    tree = fmm.Tree(x, cfg["ncrit"])
    lists = fmm.Lists(tree, cfg["theta"])
    print("gpu tree+lists %.1fs" % (time.perf_counter() - t0), flush=True)
    dt = torch.float64 if precision == "fp64" else torch.float32
    phi, g = fmm.evaluate(tree, lists, torch.tensor(q, dtype=dt, device=DEV), cfg["p"],
                          precision)
    torch.cuda.synchronize()
    return tree, lists, phi.double().cpu().numpy(), g.double().cpu().numpy()


def test_uniform_1e6_p4_all_bodies():
    cfg = W.CONFIGS["uniform-1e6-p4"]
    x = W.positions(cfg["n"], cfg["dist"])
    q = W.charges(cfg["n"], cfg["charges"])
    t0 = time.perf_counter()
    o = O.OracleFMM(x, cfg["ncrit"], cfg["theta"])
    ref = o.evaluate(q, cfg["p"])
    print("oracle %.1fs" % (time.perf_counter() - t0), flush=True)
    for precision, tol in (("mixed", 1e-5), ("fp64", 1e-12)):
        _, lists, phi, g = run_gpu(x, q, cfg, precision)
        print(precision, "e_phi", rel(phi, ref["phi"]), "e_grad", rel(g, ref["grad"]), flush=True)
        assert rel(phi, ref["phi"]) <= tol
        assert rel(g, ref["grad"]) <= tol
    tg = W.sample_targets(cfg["n"], 1000)
    dphi, dg = O.direct(x, q, tg)
    e_or = max(rel(ref["phi"][tg], dphi), rel(ref["grad"][tg], dg))
    _, _, phi, g = run_gpu(x, q, cfg, "mixed")
    assert rel(phi[tg], dphi) <= e_or + 1e-5
    assert rel(g[tg], dg) <= e_or + 1e-5


def _sample_leaves(t, ptr, nb_of, k, seed):
    leaves = np.nonzero(t["n_child"] == 0)[0]
    rng = np.random.default_rng(seed)
    pick = set(rng.choice(leaves, k, replace=False).tolist())
    rows = np.array([nb_of[ptr[a]:ptr[a + 1]].sum() for a in leaves])
    pick.update(leaves[np.argsort(rows)[-8:]].tolist())          # longest P2P rows
    pick.update(leaves[np.argsort(t["level"][leaves])[-8:]].tolist())  # deepest leaves
    return np.array(sorted(pick), dtype=np.int32)


def test_plummer_1e6_p6_sampled_leaves():
    cfg = W.CONFIGS["plummer-1e6-p6"]
    x = W.positions(cfg["n"], cfg["dist"])
    q = W.charges(cfg["n"], cfg["charges"])
    t0 = time.perf_counter()
    o = O.OracleFMM(x, cfg["ncrit"], cfg["theta"])
    t = o.tree()
    ptr, col = o.lists(O.P2P)
    leaves = _sample_leaves(t, ptr, t["n_body"][col], 48, seed=40)
    idx, rphi, rg = O.evaluate_leaves(o, q, cfg["p"], leaves)
    print("oracle sampled %d bodies in %.1fs" % (len(idx), time.perf_counter() - t0), flush=True)
    _, lists, phi, g = run_gpu(x, q, cfg, "mixed")
    assert lists.stats()["p2p_max_row_sources"] > 8192  # rows split into several chunks
    print("e_phi", rel(phi[idx], rphi), "e_grad", rel(g[idx], rg), flush=True)
    assert rel(phi[idx], rphi) <= 1e-5
    assert rel(g[idx], rg) <= 1e-5


def test_uniform_1e7_p8_direct_sum_sample():
    cfg = W.CONFIGS["uniform-1e7-p8"]
    x = W.positions(cfg["n"], cfg["dist"])
    q = W.charges(cfg["n"], cfg["charges"])
    _, lists, phi, g = run_gpu(x, q, cfg, "mixed")
    tg = W.sample_targets(cfg["n"], 1000)
    t0 = time.perf_counter()
    dphi, dg = O.direct(x, q, tg)
    print("direct sum %.1fs" % (time.perf_counter() - t0), flush=True)
    e_phi, e_grad = rel(phi[tg], dphi), rel(g[tg], dg)
    print("e_phi", e_phi, "e_grad", e_grad, lists.stats(), flush=True)
    bound = cfg["theta"] ** cfg["p"]
    assert e_phi <= bound and e_grad <= bound
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(g))
