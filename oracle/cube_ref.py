"""Data-cube fitting reference (test infrastructure only; shares no code with
the GPU library).

The paper names cube fitting, next to spectral-line fitting, as a problem the
same three steps serve once the dimensionality may change (Sec. 5, last
paragraph), and fixes no model.  The reading taken here extends the image
readings by a spectral axis:

  - a cube D[c][y][x] holds Nc spectral channels of an H x W image; channel c
    is centred at v = c (velocities in channel units), spaxel (i, j) at
    (x = j, y = i);
  - the model is one Sersic component (the profile, centre, axis ratio and
    angle of the image model) whose light carries one Gaussian emission line
    of width sigma_v, centred at the line-of-sight velocity of a thin
    rotating disk with the component's geometry:
        V(x, y) = v0 + vproj (2/pi) atan(R / rt) x' / R,   V = v0 at R = 0,
    x' the offset along the major axis and R the elliptical radius of the
    profile, vproj the projected rotation amplitude (vmax sin i, which the
    velocity field alone does not separate) and rt the turnover radius;
  - a voxel is the mean over S x S spatial and Sv spectral midpoint
    sub-samples of  I(x, y) exp(-(v - V(x, y))^2 / (2 sigma_v^2));
  - the cube is evaluated on the padded grid (spatial H + K - 1 by
    W + K - 1 from -(K - 1)/2, spectral Nc + Kl - 1 from -(Kl - 1)/2) and
    convolved with the separable kernel psf[a][b] lsf[u], keeping the valid
    part
        out[c][y][x] = sum_{u,a,b} lsf[u] psf[a][b] pad[c+Kl-1-u][y+K-1-a][x+K-1-b],
    then a constant continuum is added;
  - parameters [xc, yc, Ie, Re, n, q, phi, continuum, v0, vproj, rt, sigma_v];
  - chi^2 = sum w (d - m)^2 with w the inverse variance;
  - the fit is the Levenberg-Marquardt rule of the image fits (damping
    D = diag(max(A_ii, 1e-12 max A_jj)), lambda x10 / /10, accept iff chi^2
    drops strictly, stop on the relative chi^2 drop or the step size after
    an accepted step, a failed Cholesky counts as an iteration).

b_n is the root of P(2n, b_n) = 1/2 taken from scipy's inverse regularised
incomplete gamma function (a library routine); its derivative in n is a
central difference of that routine.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gammaincinv

NPAR = 12
# parameter slots
XC, YC, IE, RE, NS, Q, PHI, CONT, V0, VPROJ, RT, SIG = range(NPAR)
# the derivative channels of the padded cube: every parameter but the continuum
JAC_PARAMS = [XC, YC, IE, RE, NS, Q, PHI, V0, VPROJ, RT, SIG]

LM_DEFAULTS = dict(max_iter=100, lambda0=1e-3, lambda_up=10.0, lambda_down=10.0, lambda_max=1e10,
                   ftol=1e-5, xtol=1e-10)


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def bn(n: float) -> float:
    return float(gammaincinv(2.0 * n, 0.5))


def dbn(n: float, h: float = 1e-5) -> float:
    return (bn(n + h) - bn(n - h)) / (2.0 * h)


def midpoints(S: int) -> np.ndarray:
    """Sub-sample offsets (s + 1/2)/S - 1/2 inside a unit cell."""
    return (np.arange(S, dtype=np.float64) + 0.5) / S - 0.5


def _spatial_samples(H: int, W: int, K: int, S: int):
    """x, y of every spatial sub-sample of the padded grid: shape (Mh, Mw, S*S)."""
    c0 = (K - 1) // 2
    ys = np.arange(H + K - 1, dtype=np.float64) - c0
    xs = np.arange(W + K - 1, dtype=np.float64) - c0
    o = midpoints(S)
    # sub-sample (b, a): y offset o[b], x offset o[a]
    Y = ys[:, None, None, None] + o[None, None, :, None]
    X = xs[None, :, None, None] + o[None, None, None, :]
    Y, X = np.broadcast_arrays(Y, X)
    Mh, Mw = ys.size, xs.size
    return X.reshape(Mh, Mw, S * S), Y.reshape(Mh, Mw, S * S)


def _spectral_samples(Nc: int, Kl: int, Sv: int) -> np.ndarray:
    """v of every spectral sub-sample of the padded axis: shape (Mc, Sv)."""
    cl = (Kl - 1) // 2
    vc = np.arange(Nc + Kl - 1, dtype=np.float64) - cl
    return vc[:, None] + midpoints(Sv)[None, :]


def geometry(theta, X, Y):
    """Rotated offsets and elliptical radius at the points (X, Y):
    x' = dx cos phi + dy sin phi, y' = -dx sin phi + dy cos phi,
    R^2 = x'^2 + (y'/q)^2."""
    t = _f64(theta)
    dx, dy = X - t[XC], Y - t[YC]
    c, s = math.cos(t[PHI]), math.sin(t[PHI])
    xp = c * dx + s * dy
    yp = -s * dx + c * dy
    R = np.sqrt(xp * xp + (yp / t[Q]) ** 2)
    return xp, yp, R


def sersic(theta, R):
    """I = Ie exp(-b_n ((R/Re)^(1/n) - 1))."""
    t = _f64(theta)
    b = bn(t[NS])
    return t[IE] * np.exp(-b * ((R / t[RE]) ** (1.0 / t[NS]) - 1.0))


def _f_of_r(R, rt):
    """atan(R/rt)/R, its limit 1/rt at R = 0."""
    out = np.empty_like(R)
    small = R < 1e-12 * rt
    out[small] = 1.0 / rt
    out[~small] = np.arctan(R[~small] / rt) / R[~small]
    return out


def velocity(theta, xp, R):
    """Line-of-sight velocity of the disk: v0 + vproj (2/pi) atan(R/rt) x'/R."""
    t = _f64(theta)
    return t[V0] + t[VPROJ] * (2.0 / math.pi) * xp * _f_of_r(R, t[RT])


def padded_cube(theta, H: int, W: int, K: int, Nc: int, Kl: int, S: int = 5, Sv: int = 3) -> np.ndarray:
    """Sub-sample means on the padded grid, shape (Nc + Kl - 1, H + K - 1, W + K - 1)."""
    t = _f64(theta)
    X, Y = _spatial_samples(H, W, K, S)
    xp, _, R = geometry(t, X, Y)
    I = sersic(t, R)                       # (Mh, Mw, S^2)
    V = velocity(t, xp, R)
    vs = _spectral_samples(Nc, Kl, Sv)     # (Mc, Sv)
    inv2s2 = 1.0 / (2.0 * t[SIG] ** 2)
    out = np.empty((vs.shape[0], X.shape[0], X.shape[1]))
    for c in range(vs.shape[0]):
        u = vs[c][None, None, None, :] - V[..., None]          # (Mh, Mw, S^2, Sv)
        out[c] = (I[..., None] * np.exp(-u * u * inv2s2)).mean(axis=(2, 3))
    return out


def conv_valid3(pad, psf, lsf) -> np.ndarray:
    """out[c][y][x] = sum_{u,a,b} lsf[u] psf[a][b] pad[c+Kl-1-u][y+K-1-a][x+K-1-b]."""
    pad, psf, lsf = _f64(pad), _f64(psf), _f64(lsf)
    Kl, K = lsf.size, psf.shape[0]
    Mc, Mh, Mw = pad.shape
    Nc, H, W = Mc - Kl + 1, Mh - K + 1, Mw - K + 1
    out = np.zeros((Nc, H, W))
    for u in range(Kl):
        for a in range(K):
            for b in range(K):
                out += lsf[u] * psf[a, b] * pad[Kl - 1 - u:Kl - 1 - u + Nc, K - 1 - a:K - 1 - a + H,
                                                K - 1 - b:K - 1 - b + W]
    return out


def model(theta, H: int, W: int, psf, lsf, Nc: int, S: int = 5, Sv: int = 3) -> np.ndarray:
    """Steps 1-2 of a cube plus the continuum, shape (Nc, H, W)."""
    psf, lsf = _f64(psf), _f64(lsf)
    pad = padded_cube(theta, H, W, psf.shape[0], Nc, lsf.size, S, Sv)
    return conv_valid3(pad, psf, lsf) + float(_f64(theta)[CONT])


def chi2(d, w, m) -> float:
    d, w, m = _f64(d), _f64(w), _f64(m)
    return math.fsum((w * (d - m) ** 2).ravel().tolist())


def dpadded_cube(theta, H: int, W: int, K: int, Nc: int, Kl: int, S: int = 5, Sv: int = 3) -> np.ndarray:
    """Derivatives of padded_cube in the order of JAC_PARAMS, shape (11, Mc, Mh, Mw).

    Per sub-sample the value is I G with G = exp(-(v - V)^2 / (2 sigma^2)):
      d/dtheta = (dI/dtheta) G + I G (v - V)/sigma^2 dV/dtheta,   d/dsigma = I G (v - V)^2/sigma^3.
    Sersic: with u = R/Re, t = u^(1/n) and E = b_n t,
      dI/dIe = I/Ie, dI/dRe = I E/(n Re), dI/dn = I (b'_n (1 - t) + E ln(u)/n^2),
      dI/dR = -I E/(n R)   (the 1/R and ln u terms are 0 at R = 0);
    rotated offsets: dx'/dxc = -cos, dx'/dyc = -sin, dy'/dxc = sin, dy'/dyc = -cos,
      dx'/dphi = y', dy'/dphi = -x';  R dR = x' dx' + (y'/q^2) dy',  R dR/dq = -y'^2/q^3;
    velocity: V - v0 = vproj (2/pi) x' f(R) with f = atan(R/rt)/R, so
      dV/dtheta = vproj (2/pi) (f dx'/dtheta + x' f'(R) dR/dtheta),
      dV/dv0 = 1, dV/dvproj = (2/pi) x' f, dV/drt = -vproj (2/pi) x' / (rt^2 + R^2),
      f'(R) = (R rt/(rt^2 + R^2) - atan(R/rt))/R^2  (0 at R = 0).
    """
    t = _f64(theta)
    X, Y = _spatial_samples(H, W, K, S)
    xp, yp, R = geometry(t, X, Y)
    c, s = math.cos(t[PHI]), math.sin(t[PHI])
    q, n, re, rt, vp = t[Q], t[NS], t[RE], t[RT], t[VPROJ]
    b, db = bn(n), dbn(n)
    I = sersic(t, R)
    nz = R > 0.0
    Rs = np.where(nz, R, 1.0)
    u = R / re
    tt = u ** (1.0 / n)
    E = b * tt
    lnu = np.where(nz, np.log(np.where(nz, u, 1.0)), 0.0)
    dI_dR = np.where(nz, -I * E / (n * Rs), 0.0)
    # derivatives of x', y' and R R' per geometric parameter
    dxp = {XC: -c, YC: -s, PHI: yp}
    dyp = {XC: s, YC: -c, PHI: -xp}
    RdR = {k: xp * dxp[k] + (yp / (q * q)) * dyp[k] for k in (XC, YC, PHI)}
    RdR[Q] = -(yp * yp) / q ** 3
    dR = {k: np.where(nz, RdR[k] / Rs, 0.0) for k in RdR}
    dI = {k: dI_dR * dR[k] for k in dR}
    dI[IE] = I / t[IE]
    dI[RE] = I * E / (n * re)
    dI[NS] = I * (db * (1.0 - tt) + E * lnu / (n * n))
    f = _f_of_r(R, rt)
    fp = np.where(nz, (Rs * rt / (rt * rt + R * R) - np.arctan(R / rt)) / (Rs * Rs), 0.0)
    k2 = 2.0 / math.pi
    dV = {}
    for k in (XC, YC, PHI):
        dV[k] = vp * k2 * (f * dxp[k] + xp * fp * dR[k])
    dV[Q] = vp * k2 * xp * fp * dR[Q]
    dV[V0] = np.ones_like(R)
    dV[VPROJ] = k2 * xp * f
    dV[RT] = -vp * k2 * xp / (rt * rt + R * R)
    V = velocity(t, xp, R)
    vs = _spectral_samples(Nc, Kl, Sv)
    sg = t[SIG]
    out = np.zeros((len(JAC_PARAMS), vs.shape[0], X.shape[0], X.shape[1]))
    for ch in range(vs.shape[0]):
        du = vs[ch][None, None, None, :] - V[..., None]          # v - V
        G = np.exp(-du * du / (2.0 * sg * sg))
        H1 = G * du / (sg * sg)                                   # dG/dV
        for j, p in enumerate(JAC_PARAMS):
            if p == SIG:
                v = I[..., None] * G * du * du / sg ** 3
            else:
                v = np.zeros_like(G)
                if p in dI:
                    v = v + dI[p][..., None] * G
                if p in dV:
                    v = v + (I * dV[p])[..., None] * H1
            out[j, ch] = v.mean(axis=(2, 3))
    return out


def jacobian(theta, H: int, W: int, psf, lsf, Nc: int, S: int = 5, Sv: int = 3) -> np.ndarray:
    """d model / d theta, shape (12, Nc, H, W), in parameter order."""
    psf, lsf = _f64(psf), _f64(lsf)
    dp = dpadded_cube(theta, H, W, psf.shape[0], Nc, lsf.size, S, Sv)
    J = np.zeros((NPAR, Nc, H, W))
    for j, p in enumerate(JAC_PARAMS):
        J[p] = conv_valid3(dp[j], psf, lsf)
    J[CONT] = 1.0
    return J


def fit_lm(theta0, psf, lsf, d, w, S: int = 5, Sv: int = 3, lo=None, hi=None, free=None, **opts):
    """Levenberg-Marquardt fit of one cube.  Returns (theta, info)."""
    o = dict(LM_DEFAULTS)
    o.update(opts)
    t = _f64(theta0).copy()
    d, w = _f64(d), _f64(w)
    Nc, H, W = d.shape
    idx = [p for p in range(NPAR) if free is None or free[p]]
    if lo is not None:
        t = np.maximum(t, _f64(lo))
    if hi is not None:
        t = np.minimum(t, _f64(hi))
    m = model(t, H, W, psf, lsf, Nc, S, Sv)
    c2 = chi2(d, w, m)
    lam = o["lambda0"]
    nfev, njev, it = 1, 0, 0
    status, reason = 6, 5
    if c2 == 0.0:
        return t, dict(chi2=c2, lam=lam, iters=0, nfev=nfev, njev=njev, status=0, reason=3)
    need_jac = True
    A = g = None
    wf = w.ravel()
    for it in range(1, int(o["max_iter"]) + 1):
        if need_jac:
            J = jacobian(t, H, W, psf, lsf, Nc, S, Sv).reshape(NPAR, -1)[idx]
            A = (J * wf) @ J.T
            g = (J * wf) @ (d - m).ravel()
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
        delta = np.linalg.solve(L.T, np.linalg.solve(L, g))
        trial = t.copy()
        for a, p in enumerate(idx):
            v = t[p] + delta[a]
            if lo is not None:
                v = max(v, float(lo[p]))
            if hi is not None:
                v = min(v, float(hi[p]))
            trial[p] = v
        mt = model(trial, H, W, psf, lsf, Nc, S, Sv)
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
