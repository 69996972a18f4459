"""Writes tests/golden/toy_hmm_variance_curve.txt: the exact relative
variance of the marginal-likelihood estimate against data length on the
binary toy HMM of the exact-variance example (Section 4), for m = 4 filters
of M = 2 particles with every stage interacting and with none (independent
filters), each relative to one bootstrap filter of 8 particles, all with
multinomial internal resampling -- the quantities of the paper's
relative-variance figure, computed by the collision formula of Theorem 3
(Section 3.3).  Calls only oracle/.  The observation sequence is simulated
from the model with a fixed seed (the paper does not give its data).

    python tests/golden/make_toy_variance_curve.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import theorem3 as T3  # noqa: E402

LENGTHS = [1, 2, 3, 5, 10, 15, 20, 30, 40, 50, 60]


def toy_data(T, seed=231206484):
    g = np.random.default_rng(seed)
    x = int(g.integers(0, 2))
    y = []
    for t in range(T):
        if t > 0 and g.random() < 0.25:
            x = 1 - x
        y.append(x if g.random() < 0.75 else 1 - x)
    return y


def main():
    y = toy_data(max(LENGTHS))
    lines = ["# Exact relative variance Var(Zhat) / Var(Zhat of one bootstrap filter of 8 particles)",
             "# on the binary toy HMM (stay 3/4, match 3/4), m = 4 filters of M = 2, multinomial",
             "# internal resampling, by Theorem 3's collision formula (oracle/theorem3.py).",
             "# Written by tests/golden/make_toy_variance_curve.py; observations simulated with seed 231206484.",
             "observations " + " ".join(str(v) for v in y),
             "# length  independent_filters  airpf_every_stage"]
    for L in LENGTHS:
        ri = T3.relative_variance(y[:L], 4, 2, interact=False)
        ra = T3.relative_variance(y[:L], 4, 2, interact=True)
        lines.append("%d %.15g %.15g" % (L, float(ri), float(ra)))
    with open(os.path.join(HERE, "toy_hmm_variance_curve.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
