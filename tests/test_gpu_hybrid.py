"""Treecode/FMM hybrid (M2P) evaluation on the GPU against the oracle's hybrid
evaluation, element by element, and against the direct sum."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1209_3516_amd import fmm  # noqa: E402
from paper_1209_3516_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dist,n,ncrit,theta,p,m2p_max,precision,tol", [
    ("uniform", 20_000, 16, 0.5, 4, 8, "fp64", 1e-12),
    ("uniform", 20_000, 16, 0.5, 4, 8, "mixed", 1e-5),
    ("plummer", 20_000, 16, 0.45, 6, 16, "mixed", 1e-5),
    ("uniform", 12_000, 8, 0.5, 3, 64, "mixed", 1e-5),
    ("uniform", 20_000, 32, 0.4, 8, 24, "mixed", 3e-5),
    ("uniform", 20_000, 32, 0.4, 8, 24, "fp64", 1e-12),
])
def test_hybrid_matches_the_oracle(dist, n, ncrit, theta, p, m2p_max, precision, tol):
    x = W.positions(n, dist)
    q = W.charges(n, "signed")
    o = O.OracleFMM(x, ncrit, theta, m2p_max=m2p_max)
    ref = o.evaluate(q, p)
    t = fmm.Tree(x, ncrit)
    lst = fmm.Lists(t, theta, m2p_max=m2p_max)
    assert lst.stats()["m2p_entries"] > 0
    dt = torch.float64 if precision == "fp64" else torch.float32
    phi, g = fmm.evaluate(t, lst, torch.tensor(q, dtype=dt, device="cuda:0"), p, precision)
    torch.cuda.synchronize()
    phi = phi.double().cpu().numpy()
    g = g.double().cpu().numpy()
    assert _rel(phi, ref["phi"]) <= tol, _rel(phi, ref["phi"])
    assert _rel(g, ref["grad"]) <= tol, _rel(g, ref["grad"])


def test_hybrid_accuracy_against_direct_sum():
    n = 100_000
    x = W.uniform_cube(n, seed=51)
    q = W.charges(n, seed=52)
    tg = W.sample_targets(n, 1000)
    dphi, dg = fmm.direct(torch.tensor(x, device="cuda:0"), torch.tensor(q, device="cuda:0"),
                          torch.tensor(tg, device="cuda:0"))
    dphi, dg = dphi.cpu().numpy(), dg.cpu().numpy()
    t = fmm.Tree(x, 16)
    qt = torch.tensor(q, dtype=torch.float32, device="cuda:0")
    errs = {}
    for m in (0, 16):
        lst = fmm.Lists(t, 0.5, m2p_max=m)
        phi, g = fmm.evaluate(t, lst, qt, 4)
        torch.cuda.synchronize()
        errs[m] = (_rel(phi.double().cpu().numpy()[tg], dphi),
                   _rel(g.double().cpu().numpy()[tg], dg))
    print("pure", errs[0], "hybrid", errs[16])
    assert errs[16][0] <= errs[0][0] * 1.05 and errs[16][1] <= errs[0][1] * 1.05


def test_autotune_returns_the_fastest_option():
    from paper_1209_3516_amd import tuning

    x = W.uniform_cube(30_000, seed=61)
    q = W.charges(30_000, seed=62)
    best, rows = tuning.autotune(x, q, 4, 0.5, ncrits=(16, 64), m2p_values=(0, 4), reps=3,
                                 n_targets=200)
    assert len(rows) == 4 and best["eval_ms"] == min(r["eval_ms"] for r in rows)
    for r in rows:
        assert r["e_phi"] < 1e-2 and r["e_grad"] < 1e-2
        assert (r["m2p_entries"] > 0) == (r["m2p_max"] > 0)
