"""The oracle still reproduces the frozen output written by tests/golden/make_golden.py."""
import json
import os

import numpy as np
import pytest

from tests.golden import make_golden

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_small.json")


@pytest.mark.parametrize("name", ["uniform-1000", "plummer-1000"])
def test_oracle_matches_frozen_output(name):
    with open(GOLDEN) as f:
        g = json.load(f)[name]
    r = make_golden.run_case(g["case"])
    want = g["result"]
    for k in ("num_cells", "p2p_nnz", "m2l_nnz", "lists_sha256"):
        assert r[k] == want[k], k
    np.testing.assert_allclose(r["phi_first8"], want["phi_first8"], rtol=1e-12)
    np.testing.assert_allclose(r["grad_first8"], want["grad_first8"], rtol=1e-12, atol=1e-12)
    assert r["e_phi"] == pytest.approx(want["e_phi"], rel=1e-6)
    assert r["e_grad"] == pytest.approx(want["e_grad"], rel=1e-6)
