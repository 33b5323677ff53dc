"""Multi-start reference (test infrastructure only; shares no code with the
GPU library): the start set of a single-Sersic guess and the per-group
choice of the best fit.

Start k of a guess theta0 = (x0, y0, Ie, Re, n, q, phi, sky): 0 unchanged;
1 n = 1 and Re x 1.5; 2 n = 4 and Re x 0.7; 3 phi + pi/2 mod pi.
Best member of a group: lowest chi^2 among converged members (status 0),
among all members if none converged; ties and NaN resolved towards the
lowest stamp index / never chosen.
"""
from __future__ import annotations

import math

import numpy as np


def expand_starts(theta0, n_starts):
    th = np.asarray(theta0, np.float64).reshape(-1, 8)
    out = []
    for t in th:
        for k in range(n_starts):
            s = t.copy()
            if k == 1:
                s[4], s[3] = 1.0, s[3] * 1.5
            elif k == 2:
                s[4], s[3] = 4.0, s[3] * 0.7
            elif k == 3:
                s[6] = math.fmod(s[6] + math.pi / 2, math.pi)
                if s[6] < 0:
                    s[6] += math.pi
            out.append(s)
    return np.array(out)


def group_best(groups, chi2, status):
    """groups: list of member index lists (increasing).  Returns the chosen index per group."""
    picks = []
    for members in groups:
        pick = None
        for only_ok in (True, False):
            best = math.inf
            for s in members:
                if only_ok and status[s] != 0:
                    continue
                c = chi2[s]
                if c < best:
                    best, pick = c, s
            if pick is not None:
                break
        picks.append(members[0] if pick is None else pick)
    return np.array(picks)
