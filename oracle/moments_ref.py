"""FP64 reference of the image-moment default starting point of a
single-Sersic fit (test infrastructure only; shares no code with the GPU
library).

Per stamp d (H x W, pixel (row i, col j) centred on (x = j, y = i)):
  sky = median of the outer frame of 4 pixels, s = RMS of the frame about sky;
  v   = (d - sky) * clamp((d - sky)/s - 2, 0, 1);
  centre = v-weighted mean position; q, phi from the eigen-decomposition of
  the v-weighted covariance (q = sqrt(minor/major), phi = angle of the major
  axis from +x, in [0, pi)), q clamped to [0.05, 1];
  Re = root of C(r) = sum(v)/2 with C(r) = sum_p v_p clamp(r - r_p + 1/2, 0, 1),
  r_p the elliptical radius of pixel p about the centre (axes q, phi);
  n = 2, Ie = F / (total flux of a unit-Ie n = 2 profile of that Re and q),
  F = sum(d - sky) over the stamp, at least 1e-3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq

from . import gfo

BORDER = 4


def frame_mask(H, W, border=BORDER):
    m = np.ones((H, W), bool)
    m[border:H - border, border:W - border] = False
    return m


def weights(d, sky, s):
    e = d - sky
    return e * np.clip(e / s - 2.0, 0.0, 1.0) if s > 0 else np.zeros_like(e)


def curve_of_growth(r, v, rp):
    return float(np.sum(v * np.clip(r - rp + 0.5, 0.0, 1.0)))


def sersic_total_flux(ie, re, n, q):
    b = gfo.bn(n)
    return 2 * math.pi * n * re * re * q * ie * math.exp(b) * b ** (-2 * n) * math.gamma(2 * n)


def guess(d):
    d = np.asarray(d, np.float64)
    H, W = d.shape
    fr = d[frame_mask(H, W)]
    sky = float(np.median(fr))
    s = float(np.sqrt(np.mean((fr - sky) ** 2)))
    v = weights(d, sky, s)
    F = float(np.sum(d - sky))
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    s0 = float(v.sum())
    if s0 <= 0:
        xc, yc, q, phi, re = W / 2, H / 2, 1.0, 0.0, 2.0
    else:
        xc, yc = float((v * xx).sum() / s0), float((v * yy).sum() / s0)
        dx, dy = xx - xc, yy - yc
        cov = np.array([[(v * dx * dx).sum(), (v * dx * dy).sum()],
                        [(v * dx * dy).sum(), (v * dy * dy).sum()]]) / s0
        lam, vec = np.linalg.eigh(cov)          # ascending eigenvalues
        q = float(np.clip(math.sqrt(max(lam[0], 0.0) / lam[1]), 0.05, 1.0)) if lam[1] > 0 else 1.0
        phi = float(np.mod(math.atan2(vec[1, 1], vec[0, 1]), math.pi))
        xp = dx * math.cos(phi) + dy * math.sin(phi)
        yp = (-dx * math.sin(phi) + dy * math.cos(phi)) / q
        rp = np.sqrt(xp * xp + yp * yp)
        half = 0.5 * s0
        rmax = float(rp.max()) + 1.0
        re = max(brentq(lambda r: curve_of_growth(r, v, rp) - half, 0.0, rmax, xtol=1e-13, rtol=1e-14), 0.1)
    ie = max(F / sersic_total_flux(1.0, re, 2.0, q), 1e-3)
    return np.array([xc, yc, ie, re, 2.0, q, phi, sky])
