"""The oracle still reproduces its recorded C1 values (tests/golden/c1_oracle.json,
written by tests/golden/make_golden.py from the oracle alone)."""
import json
import os

import numpy as np

from oracle import rtu_oracle as O
from tests.golden.make_golden import c1_with_mock_image


def test_oracle_reproduces_c1_fixture():
    with open(os.path.join(os.path.dirname(__file__), "golden", "c1_oracle.json")) as f:
        g = json.load(f)
    p = c1_with_mock_image()
    p.lens[0] = (p.lens[0].astype(np.float64) + np.array([0.01, 0.005, -0.004, 0.003, -0.002, 0.001, 0.002])).astype(np.float32)
    r = O.loss_grad_problem(p, 0)
    assert abs(float(r["loss"].detach()) - g["loss"]) <= 1e-10 * abs(g["loss"])
    assert np.allclose(r["grad_lens"].numpy(), g["grad_lens"], rtol=1e-9, atol=1e-9)
    assert np.allclose(r["grad_ps"].numpy(), g["grad_ps"], rtol=1e-9, atol=1e-9)
    assert abs(float(r["grad_latent"].sum()) - g["grad_latent_sum"]) < 1e-8 * max(1, abs(g["grad_latent_sum"]))
    assert r["status"] == g["status"]
