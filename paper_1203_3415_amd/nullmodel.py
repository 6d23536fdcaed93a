"""Motif significance against a null-model ensemble (host side).

The paper's step (iii) (Section "Implementation"): compare each class count
of the real graph with its distribution over randomised graphs.  The counts
come from the GPU batch census; this module only forms the z-scores, from
exact integer sums so the result does not depend on summation order.
"""
from __future__ import annotations

import numpy as np


def zscores(hists: np.ndarray, real_row: int = 0) -> np.ndarray:
    """z_c = (N_real,c - mean_c) / sd_c over all rows except `real_row`, with
    the sample standard deviation (ddof = 1); NaN where sd = 0 or fewer than
    two randomised graphs."""
    h = np.asarray(hists)
    real = [int(x) for x in h[real_row]]
    rows = [i for i in range(h.shape[0]) if i != real_row]
    cnt = len(rows)
    z = np.full(h.shape[1], np.nan)
    if cnt < 2:
        return z
    for c in range(h.shape[1]):
        col = [int(h[i, c]) for i in rows]
        s1 = sum(col)
        s2 = sum(v * v for v in col)
        var_num = cnt * s2 - s1 * s1          # = cnt (cnt - 1) * sample variance, exact
        if var_num <= 0:
            continue
        from fractions import Fraction
        mean = Fraction(s1, cnt)
        var = Fraction(var_num, cnt * (cnt - 1))
        z[c] = float(real[c] - mean) / float(var) ** 0.5
    return z
