"""Random-walk Metropolis reference (test infrastructure only; shares no code
with the GPU library).

One chain per parameter vector; target exp(-chi2/2) with a flat prior on the
box [lo, hi]; proposal theta' = theta + scale z.  Chain c at step t draws its
normals from Philox4x64-10 blocks with counter (b, c, step0 + t, stream),
b = 0..3 (Box-Muller pairs in word order), and its acceptance uniform from
word 0 of block b = 4; it accepts iff ln u < -(chi2' - chi2)/2.
"""
from __future__ import annotations

import math

import numpy as np

from .philox_ref import normals, raw_blocks, uniform24


def run(theta0, scale, n_steps, chi2_fn, key, stream=0, step0=0, lo=None, hi=None):
    """theta0, scale: [n_chains, P].  chi2_fn(chain, theta) -> chi^2 (FP64).
    Returns states [n_steps, n_chains, P] (after each step), chi2 [n_steps,
    n_chains], accepted [n_steps, n_chains] (bool) and margin [n_steps,
    n_chains] = |ln u + (chi2' - chi2)/2| (inf when theta' left the box)."""
    th = np.array(theta0, np.float64)
    nc, P = th.shape
    c2 = np.array([chi2_fn(c, th[c]) for c in range(nc)])
    states = np.empty((n_steps, nc, P))
    chis = np.empty((n_steps, nc))
    acc = np.zeros((n_steps, nc), bool)
    margin = np.full((n_steps, nc), np.inf)
    for t in range(n_steps):
        for c in range(nc):
            ctr = [0, c, step0 + t, stream]
            z = normals(key, ctr, P)
            prop = th[c] + scale[c] * z
            inside = True
            if lo is not None and np.any(prop < lo[c]):
                inside = False
            if hi is not None and np.any(prop > hi[c]):
                inside = False
            if inside:
                cp = chi2_fn(c, prop)
                u = uniform24(raw_blocks(key, [4, c, step0 + t, stream], 1))[0, 0]
                lhs, rhs = math.log(u), -0.5 * (cp - c2[c])
                margin[t, c] = abs(lhs - rhs)
                if lhs < rhs:
                    th[c] = prop
                    c2[c] = cp
                    acc[t, c] = True
            states[t, c] = th[c]
            chis[t, c] = c2[c]
    return states, chis, acc, margin
