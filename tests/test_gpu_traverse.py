"""Dual tree traversal on the GPU: lists identical bit for bit to the host
traversal's (which equal the oracle's, tests/test_lib_host.py), and the
evaluation with either lists identical bit for bit."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1209_3516_amd import fmm  # noqa: E402
from paper_1209_3516_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _points(kind):
    if kind == "uniform":
        return W.uniform_cube(50_000, seed=90)
    if kind == "plummer":
        return W.plummer(50_000, seed=91)
    if kind == "dup":
        b = W.uniform_cube(3000, seed=92)
        return np.concatenate([b, b[:1000], np.tile([[0.5, 0.5, 0.5]], (300, 1))])
    if kind == "single":
        return W.uniform_cube(20, seed=93)
    if kind == "one":
        return np.array([[0.1, 0.2, 0.3]])


@pytest.mark.parametrize("kind", ["uniform", "plummer", "dup", "single", "one"])
@pytest.mark.parametrize("ncrit,theta,leaf_first", [(32, 0.4, False), (8, 0.6, True),
                                                     (64, 0.2, False)])
def test_gpu_lists_equal_host_lists(kind, ncrit, theta, leaf_first):
    x = _points(kind)
    t = fmm.Tree(x, ncrit)
    host = fmm.Lists(t, theta, leaf_first=leaf_first)
    gpu = fmm.Lists(t, theta, leaf_first=leaf_first, device=True)
    for k in (fmm.FMM_P2P, fmm.FMM_M2L):
        hp, hc = host.csr(k)
        gp, gc = gpu.csr(k)
        np.testing.assert_array_equal(hp, gp)
        np.testing.assert_array_equal(hc, gc)
    assert host.stats()["p2p_pairs"] == gpu.stats()["p2p_pairs"]


def test_evaluation_with_gpu_lists_is_identical():
    x = W.uniform_cube(200_000, seed=94)
    q = torch.tensor(W.charges(200_000, seed=95), dtype=torch.float32, device="cuda:0")
    t = fmm.Tree(x, 64)
    a = fmm.evaluate(t, fmm.Lists(t, 0.4), q, 4)
    b = fmm.evaluate(t, fmm.Lists(t, 0.4, device=True), q, 4)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_gpu_traversal_full_size():
    x = W.uniform_cube(1_000_000)
    t = fmm.Tree(x, 64)
    fmm.Lists(t, 0.4, device=True)  # warm-up (device upload of the tree)
    t0 = time.perf_counter()
    host = fmm.Lists(t, 0.4)
    t1 = time.perf_counter()
    gpu = fmm.Lists(t, 0.4, device=True)
    t2 = time.perf_counter()
    print("host traversal %.1f ms, GPU traversal %.1f ms" % (1e3 * (t1 - t0), 1e3 * (t2 - t1)))
    for k in (fmm.FMM_P2P, fmm.FMM_M2L):
        np.testing.assert_array_equal(host.csr(k)[1], gpu.csr(k)[1])
