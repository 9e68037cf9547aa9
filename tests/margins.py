"""Margin-rejection step of the input generator (test infrastructure).

Clusters whose decision lies within eps of a threshold in double
(oracle.nf_margins: the neighbour finder's window tests, D cut and best-vs-
second gap; with constructor=True also the tracklet constructor's chi2 cut and
propagation guards, and its best-vs-second chi2 gap within 1e-3) are re-drawn -- moved by a seeded Gaussian jitter of
0.01 cm, a sub-stream per (seed, round) -- until none is left (at most
max_rounds rounds).  On such inputs the float and double decisions agree.
"""
import numpy as np

import oracle


def margin_clean(cs, eps=1e-5, seed=0, max_rounds=10, jitter=0.01, constructor=True):
    """Returns (cs, rounds, redrawn) with cs modified in place."""
    y = np.array(cs.y, dtype=np.float32, copy=True)
    z = np.array(cs.z, dtype=np.float32, copy=True)
    cs.y, cs.z = y, z
    redrawn = 0
    for rnd in range(max_rounds + 1):
        bad = np.nonzero(oracle.nf_margins(cs, eps, constructor=constructor))[0]
        if len(bad) == 0:
            return cs, rnd, redrawn
        if rnd == max_rounds:
            break
        rng = np.random.default_rng([seed, rnd])
        y[bad] = (y[bad] + rng.normal(0.0, jitter, len(bad))).astype(np.float32)
        z[bad] = (z[bad] + rng.normal(0.0, jitter, len(bad))).astype(np.float32)
        redrawn += len(bad)
    raise RuntimeError(f"{len(bad)} clusters still within the margin after {max_rounds} rounds")
