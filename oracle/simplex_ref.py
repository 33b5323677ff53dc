"""Nelder-Mead reference (Nelder & Mead 1965) for one stamp (test
infrastructure only; shares no code with the GPU library).

Coefficients: reflection 1, expansion 2, contraction 1/2, shrink 1/2.
Initial simplex: x0 and x0 + step_j e_j, clipped into [lo, hi]; every new
point is clipped too.  Ordering by (f, index): the best is the lowest value
(ties to the lower index), the worst the highest (ties to the higher index),
the second worst the highest among the others.  Each iteration: reflect;
if f_r < f_best try the expansion (keep the better of x_e, x_r); if
f_best <= f_r < f_second-worst keep x_r; otherwise contract (outside, kept if
f_c <= f_r, when f_r < f_worst; inside, kept if f_c < f_worst, otherwise) or
shrink every vertex towards the best.  Stop when 2 (f_w - f_b) <= ftol
(|f_w| + |f_b|) + 1e-300 at the start of an iteration, or after max_iter
iterations.  NaN counts as +infinity.
"""
from __future__ import annotations

import math

import numpy as np


def _order(f):
    b = w = 0
    for v in range(1, len(f)):
        if f[v] < f[b]:
            b = v
        if f[v] >= f[w]:
            w = v
    sw = 1 if w == 0 else 0
    for v in range(len(f)):
        if v != w and f[v] >= f[sw]:
            sw = v
    return b, w, sw


def minimize(fun, x0, step, lo=None, hi=None, ftol=1e-8, max_iter=2000):
    """Returns (x_best, f_best, iters, nfev, converged, trace, margins).
    margins: for every comparison that chose a branch, (number of evaluations
    so far, |a - b| / max(|a|, |b|))."""
    x0 = np.asarray(x0, np.float64)
    P = x0.size
    lo = np.full(P, -np.inf) if lo is None else np.asarray(lo, np.float64)
    hi = np.full(P, np.inf) if hi is None else np.asarray(hi, np.float64)
    clip = lambda x: np.minimum(np.maximum(x, lo), hi)
    trace, margins = [], []

    def f(x):
        v = float(fun(x))
        v = math.inf if math.isnan(v) else v
        trace.append(v)
        return v

    def cmp(a, b):
        if math.isfinite(a) and math.isfinite(b):
            margins.append((len(trace), abs(a - b) / max(abs(a), abs(b), 1e-300)))

    X = [clip(x0.copy())]
    for j in range(P):
        x = x0.copy()
        x[j] += step[j]
        X.append(clip(x))
    X = np.array(X)
    F = np.array([f(x) for x in X])
    iters = 0
    while True:
        b, w, sw = _order(F)
        if 2.0 * (F[w] - F[b]) <= ftol * (abs(F[w]) + abs(F[b])) + 1e-300:
            return X[b].copy(), F[b], iters, len(trace), True, trace, margins
        if iters >= max_iter:
            return X[b].copy(), F[b], iters, len(trace), False, trace, margins
        iters += 1
        c = np.zeros(P)
        for v in range(P + 1):
            if v != w:
                c = c + X[v]
        c = c / P
        xr = clip(c + (c - X[w]))
        fr = f(xr)
        cmp(fr, F[b])
        if fr < F[b]:
            xe = clip(c + 2.0 * (xr - c))
            fe = f(xe)
            cmp(fe, fr)
            if fe < fr:
                X[w], F[w] = xe, fe
            else:
                X[w], F[w] = xr, fr
            continue
        cmp(fr, F[sw])
        if fr < F[sw]:
            X[w], F[w] = xr, fr
            continue
        cmp(fr, F[w])
        if fr < F[w]:
            xc = clip(c + 0.5 * (xr - c))
            fc = f(xc)
            cmp(fc, fr)
            ok = fc <= fr
        else:
            xc = clip(c + 0.5 * (X[w] - c))
            fc = f(xc)
            cmp(fc, F[w])
            ok = fc < F[w]
        if ok:
            X[w], F[w] = xc, fc
            continue
        for v in range(P + 1):
            if v != b:
                X[v] = X[b] + 0.5 * (X[v] - X[b])
                F[v] = f(X[v])
