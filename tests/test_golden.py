"""The oracle reproduces its stored fixture (written by tests/golden/make_golden.py)."""
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_logistic_c0_fixture():
    with open(os.path.join(HERE, "golden", "logistic_c0.json")) as fh:
        g = json.load(fh)
    r = oracle.ieks("logistic", [], [0.01], 0.0, 10.0, 2, 1000, max_iter=20, tol=1e-10)
    assert r["status"] == g["status"] and r["iterations"] == g["iterations"]
    m = r["mean"][g["n"]]
    assert np.abs(m - np.array(g["mean"])).max() <= 1e-12 * np.abs(g["mean"]).max()
    v = np.array([(r["sqrtcov"][n] @ r["sqrtcov"][n].T)[0, 0] for n in g["n"]])
    assert np.allclose(v, g["var_E0"], rtol=1e-9, atol=1e-300)
