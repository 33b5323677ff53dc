"""Spectral-line fitting reference (test infrastructure only; shares no code
with the GPU library).

The paper names spectral-line and cube fitting as the next problems for the
same three steps once the dimensionality is allowed to change (Sec. 5, last
paragraph), without fixing a model.  The readings taken here are the 1-D
counterparts of the image readings:
  - a spectrum has N channels; channel i is centred at x = i and its value is
    the mean of S midpoint sub-samples at x = i + (s + 1/2)/S - 1/2;
  - the model is a sum of Gaussian lines A exp(-(x - mu)^2 / (2 sigma^2))
    (A the peak, mu the centre and sigma the width, both in channels),
    evaluated on a padded axis of N + K - 1 channels that starts at channel
    -c, c = (K - 1)/2, convolved with the K-tap line-spread function keeping
    the valid part  out[i] = sum_u lsf[u] pad[i + K - 1 - u],  plus a constant
    continuum added after the convolution;
  - chi^2 = sum_i w_i (d_i - m_i)^2 with w the inverse variance;
  - parameters [A_1, mu_1, sigma_1, ..., A_L, mu_L, sigma_L, continuum];
  - the fit is the Levenberg-Marquardt rule of the image fits (damping
    D = diag(max(A_ii, 1e-12 max A_jj)), x10 / /10, accept iff chi^2 drops
    strictly, stop on the relative chi^2 drop or the step size after an
    accepted step, a failed Cholesky counts as an iteration).
"""
from __future__ import annotations

import math

import numpy as np

LM_DEFAULTS = dict(max_iter=100, lambda0=1e-3, lambda_up=10.0, lambda_down=10.0, lambda_max=1e10,
                   ftol=1e-5, xtol=1e-10)


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def padded_axis(N: int, K: int) -> np.ndarray:
    """Channel positions of the padded axis: -c .. N - 1 + c."""
    c = (K - 1) // 2
    return np.arange(N + K - 1, dtype=np.float64) - c


def subsample_offsets(S: int) -> np.ndarray:
    return (np.arange(S, dtype=np.float64) + 0.5) / S - 0.5


def lines_padded(theta, N: int, K: int, S: int) -> np.ndarray:
    """Sub-sample mean of the sum of the lines on the padded axis."""
    t = _f64(theta)
    x = padded_axis(N, K)[:, None] + subsample_offsets(S)[None, :]
    v = np.zeros_like(x)
    for k in range((t.size - 1) // 3):
        a, mu, sg = t[3 * k:3 * k + 3]
        v += a * np.exp(-(x - mu) ** 2 / (2.0 * sg * sg))
    return v.mean(axis=1)


def conv_valid(pad, lsf) -> np.ndarray:
    """out[i] = sum_u lsf[u] pad[i + K - 1 - u], i = 0 .. len(pad) - K."""
    pad, lsf = _f64(pad), _f64(lsf)
    K = lsf.size
    N = pad.size - K + 1
    out = np.zeros(N)
    for u in range(K):
        out += lsf[u] * pad[K - 1 - u:K - 1 - u + N]
    return out


def model(theta, N: int, lsf, S: int = 5) -> np.ndarray:
    lsf = _f64(lsf)
    return conv_valid(lines_padded(theta, N, lsf.size, S), lsf) + float(_f64(theta)[-1])


def chi2(d, w, m) -> float:
    d, w, m = _f64(d), _f64(w), _f64(m)
    return math.fsum((w * (d - m) ** 2).tolist())


def jacobian(theta, N: int, lsf, S: int = 5) -> np.ndarray:
    """d model / d theta, [P, N]: per line the sub-sample means of
    g, A g (x - mu)/sigma^2 and A g (x - mu)^2/sigma^3 (g the unit-peak
    Gaussian), convolved like the model; the continuum row is all ones."""
    t = _f64(theta)
    lsf = _f64(lsf)
    K = lsf.size
    x = padded_axis(N, K)[:, None] + subsample_offsets(S)[None, :]
    P = t.size
    J = np.zeros((P, N))
    for k in range((P - 1) // 3):
        a, mu, sg = t[3 * k:3 * k + 3]
        dx = x - mu
        g = np.exp(-dx * dx / (2.0 * sg * sg))
        J[3 * k] = conv_valid(g.mean(axis=1), lsf)
        J[3 * k + 1] = conv_valid((a * g * dx / (sg * sg)).mean(axis=1), lsf)
        J[3 * k + 2] = conv_valid((a * g * dx * dx / (sg ** 3)).mean(axis=1), lsf)
    J[P - 1] = 1.0
    return J


def fit_lm(theta0, lsf, d, w, S: int = 5, lo=None, hi=None, free=None, **opts):
    """Levenberg-Marquardt fit of one spectrum.  Returns (theta, info)."""
    o = dict(LM_DEFAULTS)
    o.update(opts)
    t = _f64(theta0).copy()
    d, w, lsf = _f64(d), _f64(w), _f64(lsf)
    N = d.size
    P = t.size
    idx = [p for p in range(P) if free is None or free[p]]
    if lo is not None:
        t = np.maximum(t, _f64(lo))
    if hi is not None:
        t = np.minimum(t, _f64(hi))
    m = model(t, N, lsf, S)
    c2 = chi2(d, w, m)
    lam = o["lambda0"]
    nfev, njev, it = 1, 0, 0
    status, reason = 6, 5
    if c2 == 0.0:
        return t, dict(chi2=c2, lam=lam, iters=0, nfev=nfev, njev=njev, status=0, reason=3)
    need_jac = True
    A = g = None
    for it in range(1, int(o["max_iter"]) + 1):
        if need_jac:
            J = jacobian(t, N, lsf, S)[idx]
            A = (J * w) @ J.T
            g = (J * w) @ (d - m)
            njev += 1
            need_jac = False
        dmax = max(A[a, a] for a in range(len(idx)))
        Ad = A.copy()
        for a in range(len(idx)):
            Ad[a, a] += lam * max(A[a, a], 1e-12 * dmax)
        try:
            L = np.linalg.cholesky(Ad)
        except np.linalg.LinAlgError:
            lam *= o["lambda_up"]
            if lam > o["lambda_max"]:
                status, reason = 6, 4
                break
            continue
        y = np.linalg.solve(L, g)
        delta = np.linalg.solve(L.T, y)
        trial = t.copy()
        for a, p in enumerate(idx):
            v = t[p] + delta[a]
            if lo is not None:
                v = max(v, float(lo[p]))
            if hi is not None:
                v = min(v, float(hi[p]))
            trial[p] = v
        mt = model(trial, N, lsf, S)
        c2t = chi2(d, w, mt)
        nfev += 1
        if c2t < c2:
            step = max(abs(trial[p] - t[p]) / max(abs(t[p]), 1.0) for p in idx)
            rel = (c2 - c2t) / c2t if c2t > 0.0 else 0.0
            t, m, c2 = trial, mt, c2t
            lam /= o["lambda_down"]
            need_jac = True
            if c2 == 0.0:
                status, reason = 0, 3
                break
            if rel < o["ftol"]:
                status, reason = 0, 1
                break
            if step < o["xtol"]:
                status, reason = 0, 2
                break
        else:
            lam *= o["lambda_up"]
            if lam > o["lambda_max"]:
                status, reason = 6, 4
                break
    else:
        status, reason = 6, 5
    return t, dict(chi2=c2, lam=lam, iters=it, nfev=nfev, njev=njev, status=status, reason=reason)
