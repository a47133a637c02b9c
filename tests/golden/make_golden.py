"""Writes the stored expected values under tests/golden/ from the FP64 oracle
alone (no GPU code is imported).  Run from the repository root:

    python tests/golden/make_golden.py

plain_small.json: the small plain workload (N=10,000, K=20, float64 X):
  * f at beta = 0, which the model fixes in closed form: every row has u = 0
    and contributes 0 - ln 2, the zero-mean prior contributes 0, so
    f(0) = -N ln 2 (logistic likelihood of Sec. 3.1.1, eq-loglike-binlogit);
  * the oracle's f and g at the first three seeded evaluation points, kept as a
    regression record of the oracle itself.
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    w = synth.plain_small(n_evals=3)
    rec = {"workload": "plain small N=10000 K=20 float64, prior sd 10",
           "f_at_zero_closed_form": -10_000 * math.log(2.0),
           "points": []}
    for beta in w.betas[:3]:
        f, g = oracle.logpost_grad(w.X, w.y, beta, w.prec)
        rec["points"].append({"beta": beta.tolist(), "f": f, "g": g.tolist()})
    with open(os.path.join(HERE, "plain_small.json"), "w") as fh:
        json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
