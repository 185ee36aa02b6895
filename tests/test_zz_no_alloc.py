"""fmm_evaluate_noalloc (the entry point that allocates nothing) against
fmm_evaluate, called through the C ABI: bit-identical outputs on two calls in
a row, the second with a smaller input, then the same on FP64; refusals for
an evaluation larger than the fixed buffer and for a tree that is not on the
device yet."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from tests.bounds import assert_close  # noqa: E402
from paper_1209_3516_amd import fmm  # noqa: E402
from paper_1209_3516_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def log(*a):
    print(*a, flush=True)


def _noalloc(tree, lists, q, p, precision):
    """One fmm_evaluate_noalloc call into NaN-filled outputs."""
    dt = q.dtype
    phi = torch.full((tree.n,), float("nan"), dtype=dt, device=DEV)
    grad = torch.full((tree.n, 3), float("nan"), dtype=dt, device=DEV)
    o = fmm._EvalOpts(p, fmm.FMM_FP64 if precision == "fp64" else fmm.FMM_MIXED, -1, 0)
    rc = fmm.lib().fmm_evaluate_noalloc(tree._h, lists._h, ctypes.byref(o),
                                        ctypes.c_void_p(q.data_ptr()),
                                        ctypes.c_void_p(phi.data_ptr()),
                                        ctypes.c_void_p(grad.data_ptr()), fmm._stream())
    return rc, phi, grad


def _case(dist, n, ncrit, theta, p, precision):
    x = W.positions(n, dist)
    q = W.charges(n, "positive" if dist == "plummer" else "signed")
    tree = fmm.Tree(x, ncrit)
    lists = fmm.Lists(tree, theta)
    dt = torch.float64 if precision == "fp64" else torch.float32
    qt = torch.tensor(q, dtype=dt, device=DEV)
    return x, q, tree, lists, qt


def test_noalloc_equals_fmm_evaluate_two_calls_then_smaller():
    L = fmm.lib()
    # call 1: Plummer 10^6, p = 6, mixed precision (about 108 MB of the 128 MiB buffer)
    log("case plummer N=1e6 ncrit=32 theta=0.35 p=6 mixed")
    x1, q1, t1, l1, qt1 = _case("plummer", 10 ** 6, 32, 0.35, 6, "mixed")
    log("fresh tree: the noalloc call must refuse it (not on the device yet)")
    rc, _, _ = _noalloc(t1, l1, qt1, 6, "mixed")
    assert rc == fmm.FMM_ESTATE, L.fmm_last_error()
    ref_phi, ref_g = fmm.evaluate(t1, l1, qt1, 6)  # puts tree, lists and plan on the device
    torch.cuda.synchronize()
    rc, phi, g = _noalloc(t1, l1, qt1, 6, "mixed")
    torch.cuda.synchronize()
    assert rc == fmm.FMM_OK, L.fmm_last_error()
    log("call 1 done")
    assert torch.equal(phi, ref_phi) and torch.equal(g, ref_g)
    # larger than the buffer: p = 8 on the same tree
    rc, _, _ = _noalloc(t1, l1, qt1, 8, "mixed")
    assert rc == fmm.FMM_EINVAL
    assert b"needs" in L.fmm_last_error()
    del t1, l1, qt1, ref_phi, ref_g, phi, g

    # call 2: a smaller input (uniform 3 * 10^4, p = 4), again against
    # fmm_evaluate and, through it, the oracle
    log("case uniform N=30000 ncrit=32 theta=0.5 p=4 mixed")
    x2, q2, t2, l2, qt2 = _case("uniform", 30000, 32, 0.5, 4, "mixed")
    ref_phi, ref_g = fmm.evaluate(t2, l2, qt2, 4)
    torch.cuda.synchronize()
    rc, phi, g = _noalloc(t2, l2, qt2, 4, "mixed")
    torch.cuda.synchronize()
    assert rc == fmm.FMM_OK, L.fmm_last_error()
    log("call 2 done")
    assert torch.equal(phi, ref_phi) and torch.equal(g, ref_g)
    ref = O.OracleFMM(x2, 32, 0.5).evaluate(q2, 4)
    assert_close(phi.double().cpu().numpy(), ref["phi"], 1e-5, "phi")
    assert_close(g.double().cpu().numpy(), ref["grad"], 1e-5, "grad")

    # FP64 on the same small tree (its FP64 bodies are uploaded by fmm_evaluate)
    log("case uniform N=30000 p=4 fp64")
    qd = qt2.double()
    ref_phi, ref_g = fmm.evaluate(t2, l2, qd, 4, "fp64")
    torch.cuda.synchronize()
    rc, phi, g = _noalloc(t2, l2, qd, 4, "fp64")
    torch.cuda.synchronize()
    assert rc == fmm.FMM_OK, L.fmm_last_error()
    assert torch.equal(phi, ref_phi) and torch.equal(g, ref_g)
    assert_close(phi.cpu().numpy(), ref["phi"], 1e-12, "phi fp64")
