"""Writes the stored expected values under tests/golden/ by calling only the
oracle.  The paper prints no numeric worked example (its figures carry all the
numbers), so the fixtures here are regression guards for the oracle itself;
the values they hold are pinned to the paper by tests/test_oracle_pins.py.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402


def logistic_c0():
    # logistic ODE of the experiments section: y' = y(1 - y), y0 = 0.01, t in [0, 10],
    # IWP(2), N = 1000, constant initial trajectory, stop at delta < 1e-10 or 20 iterations
    r = oracle.ieks("logistic", [], [0.01], 0.0, 10.0, 2, 1000, max_iter=20, tol=1e-10)
    idx = [0, 1, 2, 10, 100, 250, 500, 750, 999, 1000]
    return {
        "problem": "logistic y0=0.01 t=[0,10] q=2 N=1000 tol=1e-10 max_iter=20",
        "status": r["status"],
        "iterations": r["iterations"],
        "deltas": [float(x) for x in r["deltas"]],
        "n": idx,
        "mean": [[float(v) for v in r["mean"][n]] for n in idx],
        "var_E0": [float((r["sqrtcov"][n] @ r["sqrtcov"][n].T)[0, 0]) for n in idx],
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "logistic_c0.json"), "w") as fh:
        json.dump(logistic_c0(), fh, indent=1)
        fh.write("\n")
