"""Independent numpy re-statement of one PC-stable level, used to pin the oracle.

Different arithmetic from the oracle on purpose: the partial correlation is taken from the inverse
of the whole (l+2) x (l+2) block (rho = -P12 / sqrt(P11 P22)), Phi^-1 comes from scipy, and subsets
come from itertools. Only the decision rule (Fisher z <= tau, both directions) is shared, because
that is the method.
"""
import itertools
import math

import numpy as np
from scipy.stats import norm


def tau(alpha, m, l):
    return norm.ppf(1.0 - alpha / 2.0) / math.sqrt(m - l - 3)


def pcor_block(C, i, j, S):
    idx = [i, j] + list(S)
    P = np.linalg.inv(C[np.ix_(idx, idx)])
    return -P[0, 1] / math.sqrt(P[0, 0] * P[1, 1])


def zstat(rho):
    if abs(rho) >= 1.0:
        return math.inf
    return abs(math.atanh(rho))


def first_separating(C, Gp, i, j, l, m, alpha):
    """First separating S of edge (i,j) in canonical order (direction i, then j), with the z gap.

    Returns (S or None, min |z - tau| over the tests looked at)."""
    t = tau(alpha, m, l)
    gap = math.inf
    for a, b in ((i, j), (j, i)):
        cand = [k for k in np.flatnonzero(Gp[a]) if k != b]
        for S in itertools.combinations(cand, l):
            z = zstat(pcor_block(C, a, b, S))
            gap = min(gap, abs(z - t))
            if z <= t:
                return tuple(int(s) for s in S), gap
    return None, gap
