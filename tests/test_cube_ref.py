"""Pins of the data-cube reference (oracle/cube_ref.py) against library
routines, the image and line oracles, closed forms and invariants (CPU only).

* the 3-D valid convolution against scipy's N-d convolution and brute force;
* no rotation (vproj = 0): the cube is the image model times the line model
  (the two other oracles, with their own b_n, sub-sampling and padding);
* any velocity field: the spectral sum of a spaxel is sigma sqrt(2 pi) times
  the image model (the line carries the light, it does not change it);
* delta kernels, one sub-sample: the first spectral moment of a spaxel is the
  disk velocity, computed here by a complex rotation at points on the major
  and minor axes and elsewhere; the second central moment is
  sigma^2 + (Sv^2 - 1) / (12 Sv^2);
* point reflection through an integer centre mirrors the spectrum about v0;
* the analytic Jacobian against central differences (also with a sub-sample
  at R = 0);
* the fit: a linear-only fit equals weighted least squares, one damped step
  equals the step recomputed from a finite-difference Jacobian, and a
  noise-free start 10 % off recovers the truth.
"""
import math

import numpy as np
import pytest
from scipy.signal import convolve

import synth
from oracle import cube_ref as CR
from oracle import line_ref as LR

TH = np.array([10.3, 9.6, 1.5, 4.0, 1.7, 0.6, 0.5, 0.02, 11.4, 4.0, 2.5, 1.6])


def _asym_psf(K, seed):
    g = np.random.default_rng(seed)
    p = g.uniform(0.1, 1.0, (K, K))
    return p / p.sum()


def _asym_lsf(K, seed):
    g = np.random.default_rng(seed)
    p = g.uniform(0.1, 1.0, K)
    return p / p.sum()


def test_conv_valid3_against_scipy_and_brute_force():
    g = np.random.default_rng(1)
    pad = g.standard_normal((7, 6, 8))
    psf = g.standard_normal((3, 3))
    lsf = np.array([0.3, -0.5, 0.9])      # asymmetric: pins the flips
    out = CR.conv_valid3(pad, psf, lsf)
    ker = lsf[:, None, None] * psf[None, :, :]
    np.testing.assert_allclose(out, convolve(pad, ker, mode="valid", method="direct"), rtol=1e-12, atol=1e-13)
    c, y, x = 2, 1, 3
    brute = sum(lsf[u] * psf[a, b] * pad[c + 2 - u, y + 2 - a, x + 2 - b]
                for u in range(3) for a in range(3) for b in range(3))
    assert out[c, y, x] == pytest.approx(brute, rel=1e-13)


@pytest.mark.parametrize("S,Sv", [(1, 1), (3, 2), (5, 3)])
def test_no_rotation_is_image_times_line(gfo, S, Sv):
    th = TH.copy()
    th[CR.VPROJ] = 0.0
    H, W, Nc = 19, 21, 24
    psf, lsf = _asym_psf(5, 2), _asym_lsf(7, 3)
    m = CR.model(th, H, W, psf, lsf, Nc, S, Sv)
    img = gfo.model(H, W, np.r_[th[:7], 0.0], psf, S)
    line = LR.model(np.array([1.0, th[CR.V0], th[CR.SIG], 0.0]), Nc, lsf, Sv)
    ref = line[:, None, None] * img[None] + th[CR.CONT]
    np.testing.assert_allclose(m, ref, rtol=1e-9, atol=1e-12)


def test_spectral_sum_is_flux_for_any_velocity_field(gfo):
    th = TH.copy()
    th[CR.V0], th[CR.VPROJ], th[CR.RT], th[CR.SIG] = 24.2, 6.0, 3.0, 1.6
    th[CR.CONT] = 0.0
    H, W, Nc = 17, 15, 48
    psf, lsf = _asym_psf(3, 4), _asym_lsf(5, 5)
    m = CR.model(th, H, W, psf, lsf, Nc, 3, 3)
    img = gfo.model(H, W, np.r_[th[:7], 0.0], psf, 3)
    np.testing.assert_allclose(m.sum(axis=0), th[CR.SIG] * math.sqrt(2 * math.pi) * img, rtol=1e-10, atol=1e-14)
    # and the field does move the light between channels
    th0 = th.copy()
    th0[CR.VPROJ] = 0.0
    assert np.abs(m - CR.model(th0, H, W, psf, lsf, Nc, 3, 3)).max() > 1e-2 * m.max()


def _disk_velocity(th, dx, dy):
    """V from a complex rotation: z = (dx + i dy) e^{-i phi}, the disk-plane
    point (Re z, Im z / q), its radius and azimuth."""
    z = complex(dx, dy) * complex(math.cos(th[CR.PHI]), -math.sin(th[CR.PHI]))
    w = complex(z.real, z.imag / th[CR.Q])
    R = abs(w)
    if R == 0.0:
        return th[CR.V0]
    return th[CR.V0] + th[CR.VPROJ] * (2 / math.pi) * math.atan(R / th[CR.RT]) * math.cos(math.atan2(w.imag, w.real))


@pytest.mark.parametrize("phi", [0.0, math.pi / 2, 0.7])
def test_velocity_moments(phi):
    th = TH.copy()
    th[CR.XC], th[CR.YC], th[CR.PHI] = 8.0, 7.0, phi
    th[CR.V0], th[CR.VPROJ], th[CR.RT], th[CR.SIG], th[CR.CONT] = 30.0, 9.0, 2.2, 1.7, 0.0
    H, W, Nc = 15, 17, 60
    one = np.ones((1, 1))
    for Sv in (1, 3):
        m = CR.model(th, H, W, one, np.ones(1), Nc, 1, Sv)
        c = np.arange(Nc, dtype=float)[:, None, None]
        tot = m.sum(axis=0)
        mom1 = (c * m).sum(axis=0) / tot
        mom2 = ((c - mom1) ** 2 * m).sum(axis=0) / tot
        for (y, x) in [(7, 8), (7, 13), (7, 2), (3, 8), (12, 8), (2, 14), (11, 5)]:
            V = _disk_velocity(th, x - th[CR.XC], y - th[CR.YC])
            assert mom1[y, x] == pytest.approx(V, abs=1e-9), (phi, y, x)
            assert mom2[y, x] == pytest.approx(th[CR.SIG] ** 2 + (Sv * Sv - 1) / (12 * Sv * Sv), abs=1e-9)
    # closed forms on the axes (phi = 0: major axis along x)
    if phi == 0.0:
        m = CR.model(th, H, W, one, np.ones(1), Nc, 1, 1)
        c = np.arange(Nc, dtype=float)[:, None, None]
        mom1 = (c * m).sum(axis=0) / m.sum(axis=0)
        for k in (-6, -2, 1, 5):
            ref = th[CR.V0] + th[CR.VPROJ] * (2 / math.pi) * math.atan(abs(k) / th[CR.RT]) * math.copysign(1, k)
            assert mom1[7, 8 + k] == pytest.approx(ref, abs=1e-9)
            assert mom1[7 + k, 8] == pytest.approx(th[CR.V0], abs=1e-9)   # minor axis: systemic
        assert mom1[7, 8] == pytest.approx(th[CR.V0], abs=1e-9)


def test_point_reflection_mirrors_the_spectrum():
    th = TH.copy()
    th[CR.XC], th[CR.YC] = 7.0, 6.0
    th[CR.V0] = 9.0
    H, W, Nc = 13, 15, 19
    psf = synth.gaussian_psf(5, 1.1)
    x = np.arange(5) - 2.0
    lsf = np.exp(-x * x / 2.0)
    lsf /= lsf.sum()
    m = CR.model(th, H, W, psf, lsf, Nc, 3, 3)
    np.testing.assert_allclose(m, m[::-1, ::-1, ::-1], rtol=1e-11, atol=1e-14)
    assert np.abs(m - m[:, ::-1, ::-1]).max() > 1e-3 * m.max()   # not symmetric without the mirror


@pytest.mark.parametrize("centre,S,n", [((4.3, 3.6), 2, 1.7), ((4.0, 4.0), 3, 0.5)])
def test_jacobian_central_differences(centre, S, n):
    """The second case puts a sub-sample at R = 0 (n = 0.5: the profile is
    smooth there, so central differences are exact to O(h^2); for n > 0.5
    the cusp makes them converge only as h^(1/n))."""
    th = TH.copy()
    th[CR.XC], th[CR.YC] = centre
    th[CR.NS] = n
    th[CR.V0], th[CR.SIG] = 4.6, 1.3
    H, W, Nc = 9, 9, 10
    psf, lsf = _asym_psf(3, 7), _asym_lsf(3, 8)
    J = CR.jacobian(th, H, W, psf, lsf, Nc, S, 2)
    for p in range(CR.NPAR):
        h = 1e-5 * max(abs(th[p]), 1.0)
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (CR.model(tp, H, W, psf, lsf, Nc, S, 2) - CR.model(tm, H, W, psf, lsf, Nc, S, 2)) / (2 * h)
        err = np.linalg.norm(J[p] - fd) / np.linalg.norm(fd)
        assert err < 1e-6, (p, err)


def _cube_case():
    th = np.array([8.3, 7.6, 1.2, 3.0, 1.4, 0.65, 0.6, 0.01, 7.3, 3.0, 2.0, 1.4])
    H, W, Nc = 15, 16, 14
    psf, lsf = synth.gaussian_psf(3, 1.0), _asym_lsf(3, 9)
    return th, H, W, Nc, psf, lsf


def test_fit_linear_only_equals_weighted_least_squares():
    th, H, W, Nc, psf, lsf = _cube_case()
    g = np.random.default_rng(11)
    d = CR.model(th, H, W, psf, lsf, Nc, 2, 2) + 0.02 * g.standard_normal((Nc, H, W))
    w = np.full(d.shape, 1 / 0.02 ** 2)
    free = np.zeros(CR.NPAR, dtype=bool)
    free[[CR.IE, CR.CONT]] = True
    start = th.copy()
    start[CR.IE] *= 1.4
    start[CR.CONT] = 0.05
    fit, info = CR.fit_lm(start, psf, lsf, d, w, 2, 2, free=free, ftol=1e-14, xtol=1e-14)
    M1 = CR.model(np.r_[th[:2], 1.0, th[3:7], 0.0, th[8:]], H, W, psf, lsf, Nc, 2, 2).ravel()
    A = np.stack([M1, np.ones_like(M1)], axis=1) * np.sqrt(w.ravel())[:, None]
    sol = np.linalg.lstsq(A, d.ravel() * np.sqrt(w.ravel()), rcond=None)[0]
    np.testing.assert_allclose([fit[CR.IE], fit[CR.CONT]], sol, rtol=1e-8, atol=1e-10)
    np.testing.assert_array_equal(fit[~free], start[~free])


def test_one_damped_step():
    th, H, W, Nc, psf, lsf = _cube_case()
    d = CR.model(th, H, W, psf, lsf, Nc, 2, 2)
    w = np.full(d.shape, 100.0)
    start = th * np.array([1.02, 0.98, 1.3, 1.2, 0.8, 1.1, 1.15, 1.0, 1.05, 1.25, 0.85, 1.1])
    fit, info = CR.fit_lm(start, psf, lsf, d, w, 2, 2, max_iter=1)
    assert info["iters"] == 1 and info["njev"] == 1
    # the step recomputed: finite-difference Jacobian, general solve
    m0 = CR.model(start, H, W, psf, lsf, Nc, 2, 2).ravel()
    J = np.zeros((CR.NPAR, m0.size))
    for p in range(CR.NPAR):
        h = 1e-6 * max(abs(start[p]), 1.0)
        tp, tm = start.copy(), start.copy()
        tp[p] += h
        tm[p] -= h
        J[p] = (CR.model(tp, H, W, psf, lsf, Nc, 2, 2) - CR.model(tm, H, W, psf, lsf, Nc, 2, 2)).ravel() / (2 * h)
    A = (J * w.ravel()) @ J.T
    gv = (J * w.ravel()) @ (d.ravel() - m0)
    D = np.maximum(np.diag(A), 1e-12 * np.diag(A).max())
    step = np.linalg.solve(A + 1e-3 * np.diag(D), gv)
    c2_start = CR.chi2(d, w, m0.reshape(d.shape))
    c2_trial = CR.chi2(d, w, CR.model(start + step, H, W, psf, lsf, Nc, 2, 2))
    if c2_trial < c2_start:
        np.testing.assert_allclose(fit, start + step, rtol=1e-5, atol=1e-7)
        assert info["lam"] == pytest.approx(1e-4)
    else:
        np.testing.assert_array_equal(fit, start)
        assert info["lam"] == pytest.approx(1e-2)
    # undamped and unit-matrix damping land elsewhere
    for alt in (np.linalg.solve(A, gv), np.linalg.solve(A + 1e-3 * np.eye(CR.NPAR), gv)):
        assert np.abs(alt - step).max() > 1e-6 * np.abs(step).max()


def test_fit_noise_free_recovers_truth():
    th, H, W, Nc, psf, lsf = _cube_case()
    d = CR.model(th, H, W, psf, lsf, Nc, 2, 2)
    w = np.full(d.shape, 100.0)
    start = th * np.array([1.01, 0.99, 1.1, 0.9, 1.1, 0.9, 1.1, 1.0, 1.02, 0.9, 1.1, 0.9])
    start[CR.CONT] = 0.0
    fit, info = CR.fit_lm(start, psf, lsf, d, w, 2, 2, ftol=1e-14, xtol=1e-14, max_iter=200)
    assert info["status"] == 0
    np.testing.assert_allclose(fit, th, rtol=1e-6, atol=1e-8)
