import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _cases():
    with open(os.path.join(HERE, "oracle_small.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("k", range(5))
def test_oracle_matches_recorded_values(k):
    c = _cases()[k]
    st, ll, gx, gp = oracle.loglik_grad(np.array(c["x"]), np.array(c["t"]), np.array(c["params"]))
    assert st == c["status"]
    assert ll == pytest.approx(c["loglik"], rel=1e-14)
    np.testing.assert_allclose(gx, np.array(c["grad_x"]), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(gp, np.array(c["grad_params"]), rtol=1e-12, atol=1e-13)
