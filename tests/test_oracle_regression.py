"""The FP64 reference still produces the stored outputs of make_golden.py."""
import json
import os

import numpy as np
import pytest

from tests.golden import make_golden

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_regression():
    with open(os.path.join(HERE, "golden", "oracle_regression.json")) as f:
        ref = json.load(f)
    got = make_golden.compute()
    for name, v in got.items():
        r = ref[name]
        assert v["dt"] == r["dt"]
        np.testing.assert_allclose(v["J_sum"], r["J_sum"], rtol=1e-12, atol=1e-12)
        assert v["J_l2"] == pytest.approx(r["J_l2"], rel=1e-12)
        np.testing.assert_allclose(v["u0"], r["u0"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(v["offs0"], r["offs0"], rtol=1e-12, atol=1e-14)
        assert v["cell0"] == r["cell0"]
        assert v["perm_head"] == r["perm_head"]
