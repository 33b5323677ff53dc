"""Pins of the spectral-line reference (oracle/line_ref.py) against closed
forms, library routines and brute force (CPU only)."""
import math

import numpy as np
import pytest
from scipy.special import erf

import synth
from oracle import line_ref as LR


def test_padded_axis_and_offsets():
    np.testing.assert_array_equal(LR.padded_axis(5, 3), [-1, 0, 1, 2, 3, 4, 5])
    np.testing.assert_allclose(LR.subsample_offsets(5), [-0.4, -0.2, 0.0, 0.2, 0.4], atol=1e-15)
    np.testing.assert_array_equal(LR.subsample_offsets(1), [0.0])


def test_conv_valid_brute_force_and_numpy():
    g = np.random.default_rng(3)
    pad = g.standard_normal(12)
    lsf = np.array([0.1, 0.5, 0.25, 0.15, 0.0, 0.3, -0.2])  # asymmetric: pins the flip
    K = lsf.size
    out = LR.conv_valid(pad, lsf)
    brute = [sum(lsf[u] * pad[i + K - 1 - u] for u in range(K)) for i in range(pad.size - K + 1)]
    np.testing.assert_allclose(out, brute, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(out, np.convolve(pad, lsf, mode="valid"), rtol=1e-13, atol=1e-14)


def test_delta_lsf_is_identity():
    th = np.array([2.0, 10.3, 1.7, 0.4])
    for K in (1, 3, 9):
        lsf = np.zeros(K)
        lsf[(K - 1) // 2] = 1.0
        m = LR.model(th, 24, lsf, 5)
        # channel i of the output is padded channel i + c, i.e. position i
        ref = LR.lines_padded(th, 24, 1, 5) + th[-1]
        np.testing.assert_allclose(m, ref, rtol=1e-15, atol=1e-15)


def test_subsample_mean_converges_to_channel_integral():
    a, mu, sg = 3.0, 7.37, 1.2
    th = np.array([a, mu, sg, 0.0])
    exact = [a * sg * math.sqrt(math.pi / 2) * (erf((i + 0.5 - mu) / (sg * math.sqrt(2)))
                                                 - erf((i - 0.5 - mu) / (sg * math.sqrt(2)))) for i in range(16)]
    for S, tol in ((5, 2e-2), (32, 6e-4), (128, 4e-5)):
        v = LR.lines_padded(th, 16, 1, S)
        # midpoint rule: error <= h^2/24 max|f''| per unit channel, h = 1/S
        assert np.max(np.abs(v - exact)) <= a / (sg * sg) / (24 * S * S) * 1.01 + 1e-15
        assert np.max(np.abs(v - exact)) <= tol


def test_total_flux_of_a_line():
    # the channel means of a Gaussian with sigma >= 1 sum to A sigma sqrt(2 pi)
    # (Poisson summation: the error is ~exp(-2 pi^2 sigma^2))
    for a, mu, sg in ((2.0, 60.3, 1.5), (0.7, 70.0, 4.0)):
        th = np.array([a, mu, sg, 0.0])
        v = LR.lines_padded(th, 140, 1, 1)
        assert v.sum() == pytest.approx(a * sg * math.sqrt(2 * math.pi), rel=1e-12)


def test_gaussian_line_through_gaussian_lsf():
    # well-sampled Gaussian line (S = 1) through a Gaussian LSF is a Gaussian
    # with summed variances and the same flux
    a, mu, sg, sl = 1.5, 80.25, 3.0, 2.0
    K = 41
    x = np.arange(K) - (K - 1) / 2
    lsf = np.exp(-x * x / (2 * sl * sl)) / (sl * math.sqrt(2 * math.pi))
    m = LR.model(np.array([a, mu, sg, 0.0]), 160, lsf, 1)
    s2 = math.sqrt(sg * sg + sl * sl)
    ref = a * sg / s2 * np.exp(-(np.arange(160) - mu) ** 2 / (2 * s2 * s2))
    np.testing.assert_allclose(m, ref, atol=1e-7 * a)


def test_chi2_self_and_fsum():
    g = np.random.default_rng(5)
    d = g.standard_normal(300)
    w = g.uniform(0.5, 2.0, 300)
    assert LR.chi2(d, w, d) == 0.0
    m = d + g.standard_normal(300) * 1e-3
    assert LR.chi2(d, w, m) == math.fsum(w * (d - m) ** 2)


def test_jacobian_against_central_differences():
    sp = synth.line_spectrum(synth.rng(11), 64, 2, 0, 11)
    th = sp.truth.copy()
    th[1], th[4] = 20.3, 41.7
    J = LR.jacobian(th, 64, sp.lsf, 3)
    for p in range(th.size):
        h = 1e-6 * max(abs(th[p]), 1.0)
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (LR.model(tp, 64, sp.lsf, 3) - LR.model(tm, 64, sp.lsf, 3)) / (2 * h)
        np.testing.assert_allclose(J[p], fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max(), err_msg=str(p))


def test_lm_linear_case_is_least_squares():
    # centres and widths fixed: the model is linear in A_k and the continuum
    sp = synth.line_spectrum(synth.rng(12), 128, 2, 0, 12)
    m0 = LR.model(sp.truth, 128, sp.lsf, 5)
    d, w = synth.add_noise_1d(m0, 0.05, 99)
    free = np.array([1, 0, 0, 1, 0, 0, 1], bool)
    start = sp.truth.copy()
    start[[0, 3, 6]] = [1.0, 1.0, 0.0]
    fit, info = LR.fit_lm(start, sp.lsf, d, w, 5, free=free, ftol=1e-14, xtol=1e-14, max_iter=200)
    J = LR.jacobian(sp.truth, 128, sp.lsf, 5)[[0, 3, 6]]
    base = LR.model(np.where(free, 0.0, sp.truth), 128, sp.lsf, 5)
    sol = np.linalg.lstsq((J * np.sqrt(w)).T, np.sqrt(w) * (d - base), rcond=None)[0]
    np.testing.assert_allclose(fit[[0, 3, 6]], sol, rtol=1e-7)
    np.testing.assert_array_equal(fit[~free], sp.truth[~free])


def test_lm_truth_start_and_noise_free_recovery():
    sp = synth.line_spectrum(synth.rng(13), 256, 3, 0, 13)
    m0 = LR.model(sp.truth, 256, sp.lsf, 5)
    w = np.ones(256)
    fit, info = LR.fit_lm(sp.truth, sp.lsf, m0, w, 5)
    assert info["status"] == 0 and info["reason"] == 3 and info["iters"] == 0
    lo, hi = synth.line_bounds(3, 256)
    fit, info = LR.fit_lm(sp.start, sp.lsf, m0, w, 5, lo=lo, hi=hi, ftol=1e-15, xtol=1e-13, max_iter=300)
    np.testing.assert_allclose(fit, sp.truth, rtol=1e-6, atol=1e-7)
    assert np.all(fit >= lo) and np.all(fit <= hi)
