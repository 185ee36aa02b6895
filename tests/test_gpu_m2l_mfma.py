"""GPU parity of box-centred trees and of the batched M2L on the matrix cores
(FMM_EVAL_M2L_MFMA) against the FP64 oracle with the same geometry.

* full evaluation, entry-by-entry M2L and batched M2L, mixed precision:
  1e-5 (p <= 6) and 3e-5 (p = 8, FP64 top levels) relative L2 plus the
  per-body bound (tests/bounds.py), on uniform and Plummer inputs, p = 1..8;
* the locals right after M2L (FMM_EVAL_KEEP_STAGES), row by row against the
  oracle's L after M2L, for both M2L kernels: what the batched product itself
  computes, with the FP64 top levels of p = 8 kept apart;
* the batched and the entry-by-entry M2L on the same lists agree with each
  other to FP32 rounding;
* refusals: a tree without box centres, FP64 precision, a target range.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from tests.bounds import assert_close, rel  # noqa: E402
from paper_1209_3516_amd import fmm  # noqa: E402
from paper_1209_3516_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [
    # name, dist, n, ncrit, theta, p
    ("uniform-20000-p4", "uniform", 20_000, 32, 0.4, 4),
    ("plummer-20000-p6", "plummer", 20_000, 16, 0.35, 6),
    ("uniform-30000-p8", "uniform", 30_000, 64, 0.3, 8),
    ("uniform-3000-p1", "uniform", 3_000, 16, 0.5, 1),
    ("plummer-5000-p3", "plummer", 5_000, 8, 0.5, 3),
    ("uniform-6000-p5", "uniform", 6_000, 12, 0.45, 5),
    ("plummer-6000-p7", "plummer", 6_000, 10, 0.35, 7),
]


def tol(p):
    return 3e-5 if p >= 8 else 1e-5


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_box_centred_evaluation_and_batched_m2l_match_oracle(case):
    name, dist, n, ncrit, theta, p = case
    print("case", name, flush=True)
    x = W.positions(n, dist)
    q = W.charges(n, "signed")
    ref = O.OracleFMM(x, ncrit, theta, box_centres=True).evaluate(q, p)
    t = fmm.Tree(x, ncrit, box_centres=True)
    lst = fmm.Lists(t, theta)
    qt = torch.tensor(q, dtype=torch.float32, device=DEV)
    out = {}
    for mfma in (False, True):
        phi, g = fmm.evaluate(t, lst, qt, p, m2l_mfma=mfma)
        torch.cuda.synchronize()
        phi, g = phi.double().cpu().numpy(), g.double().cpu().numpy()
        assert_close(phi, ref["phi"], tol(p), "phi mfma=%s" % mfma)
        assert_close(g, ref["grad"], tol(p), "grad mfma=%s" % mfma)
        out[mfma] = (phi, g)
    # the two M2L kernels differ by FP32 rounding only
    assert rel(out[True][0], out[False][0]) <= 0.5 * tol(p)
    assert rel(out[True][1], out[False][1]) <= 0.5 * tol(p)


@pytest.mark.parametrize("dist,p", [("uniform", 4), ("plummer", 6), ("uniform", 8)])
def test_batched_m2l_locals_match_oracle_row_by_row(dist, p):
    n = 8000
    x = W.positions(n, dist)
    q = W.charges(n, "signed")
    o = O.OracleFMM(x, 16, 0.4, box_centres=True)
    ref = o.evaluate(q, p, staged=True)["L_m2l"]
    t = fmm.Tree(x, 16, box_centres=True)
    lst = fmm.Lists(t, 0.4)
    qt = torch.tensor(q, dtype=torch.float32, device=DEV)
    ex_lib = [tuple(r) for r in fmm.term_exponents(p).tolist()]
    ex_or = [tuple(r) for r in O.term_exponents(p).tolist()]
    perm = [ex_lib.index(e) for e in ex_or]
    level = o.tree()["level"]
    top = 3 if p >= 8 else -1  # FP64-accumulated levels (entry by entry in both modes)
    for mfma in (False, True):
        fmm.evaluate(t, lst, qt, p, keep_stages=True, m2l_mfma=mfma)
        torch.cuda.synchronize()
        got = fmm.copy_expansions(lst, 1, p)[:, perm]
        scale = np.max(np.abs(ref), axis=1) + 1e-300
        err = np.max(np.abs(got - ref), axis=1) / scale
        rows = level > top
        assert np.max(err[rows]) <= 1e-4, "mfma=%s worst row %.2e" % (mfma, np.max(err[rows]))
        assert np.median(err[rows]) <= 1e-5


def test_batched_m2l_refusals():
    x = W.uniform_cube(4000)
    q = torch.tensor(W.charges(4000), dtype=torch.float32, device=DEV)
    plain = fmm.Tree(x, 16)
    lp = fmm.Lists(plain, 0.4)
    with pytest.raises(fmm.FMMError) as e:
        fmm.evaluate(plain, lp, q, 4, m2l_mfma=True)
    assert e.value.code == fmm.FMM_EINVAL
    box = fmm.Tree(x, 16, box_centres=True)
    lb = fmm.Lists(box, 0.4)
    with pytest.raises(fmm.FMMError) as e:
        fmm.evaluate(box, lb, q.double(), 4, "fp64", m2l_mfma=True)
    assert e.value.code == fmm.FMM_EINVAL
    bounds = fmm.partition(box, lb, 2)
    with pytest.raises(fmm.FMMError) as e:
        fmm.evaluate(box, lb, q, 4, m2l_mfma=True, body_range=(bounds[0], bounds[1]))
    assert e.value.code == fmm.FMM_EINVAL
    # still usable afterwards
    phi, _ = fmm.evaluate(box, lb, q, 4, m2l_mfma=True)
    torch.cuda.synchronize()
    assert torch.isfinite(phi).all()
