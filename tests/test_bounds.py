"""The error measures of the parity tests (tests/bounds.py), checked on the
oracle's own output with mistakes planted in it on the CPU."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1209_3516_amd import workloads as W
from tests.bounds import PER_BODY, assert_close, per_body_ratio, rel


@pytest.fixture(scope="module")
def ref():
    x = W.uniform_cube(20_000, seed=61)
    q = W.charges(20_000, seed=62)
    o = O.OracleFMM(x, 32, 0.4)
    return o, o.evaluate(q, 4)


def test_exact_values_pass(ref):
    _, r = ref
    assert_close(r["phi"], r["phi"], 1e-12)
    assert_close(r["grad"], r["grad"], 1e-12)


def test_error_confined_to_one_leaf_is_caught(ref):
    """A 1.5e-4 relative error on the bodies of one leaf moves the global norm by
    well under 1e-5 but breaks the per-body bound."""
    o, r = ref
    t = o.tree()
    leaf = int(np.nonzero(t["n_child"] == 0)[0][7])
    b0, nb = int(t["body_begin"][leaf]), int(t["n_body"][leaf])
    users = t["perm"][b0:b0 + nb]
    for key in ("phi", "grad"):
        bad = r[key].copy()
        bad[users] *= 1.0 + 1.5e-4
        assert rel(bad, r[key]) < 1e-5
        assert per_body_ratio(bad, r[key]) > PER_BODY * 1e-5
        with pytest.raises(AssertionError):
            assert_close(bad, r[key], 1e-5)


def test_uniform_rounding_passes_and_wrong_values_fail(ref):
    _, r = ref
    f32 = r["grad"].astype(np.float32).astype(np.float64)
    assert_close(f32, r["grad"], 1e-6)
    swapped = r["grad"][:, [1, 0, 2]]  # transposed components
    with pytest.raises(AssertionError):
        assert_close(swapped, r["grad"], 1e-5)


def test_floor_for_values_near_zero():
    """A body whose exact value is about zero is held to the rms scale, not to
    its own magnitude."""
    ref = np.array([1.0, -1.0, 1e-12, 2.0])
    got = ref + np.array([0.0, 0.0, 1e-6, 0.0])
    assert per_body_ratio(got, ref) == pytest.approx(1e-6 / np.sqrt(np.mean(ref ** 2)))
