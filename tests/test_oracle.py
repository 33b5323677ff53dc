"""Pins of the FP64 oracle against things other than itself.

Each check uses a library routine (scipy.special, scipy.signal, numpy.linalg),
a closed form, a geometric special case or brute force on tiny inputs, so
that a dropped term, a wrong sign, a transposed operand or a wrong constant
anywhere in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.signal
import scipy.special as sp

import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------- b_n (D3) ---
@pytest.mark.parametrize("a,x", [(0.4, 0.01), (0.4, 2.0), (1.0, 1.0), (3.3, 2.1), (3.3, 12.1), (12.0, 11.5),
                                 (20.0, 19.7), (20.0, 40.0), (5.0, 0.3)])
def test_gammp_matches_scipy(gfo, a, x):
    assert gfo.gammp(a, x) == pytest.approx(sp.gammainc(a, x), rel=1e-13, abs=1e-300)


@pytest.mark.parametrize("n", np.concatenate([np.linspace(0.2, 10.0, 50), [0.5, 1, 2.5, 4, 6]]))
def test_bn_is_median_of_gamma(gfo, n):
    # b_n solves Gamma(2n) = 2 gamma(2n, b_n): the inverse regularised gamma at 1/2.
    assert gfo.bn(n) == pytest.approx(sp.gammaincinv(2 * n, 0.5), rel=1e-13)


def test_bn_known_values(gfo):
    # b_0.5 = ln 2 exactly (the Gaussian); the others are tabulated in the literature.
    assert gfo.bn(0.5) == pytest.approx(math.log(2.0), rel=1e-14)
    for n, b in [(1.0, 1.67834699), (2.5, 4.67090888), (4.0, 7.66924944), (6.0, 11.66836315)]:
        assert gfo.bn(n) == pytest.approx(b, abs=6e-9)


@pytest.mark.parametrize("n", [0.25, 0.5, 1.0, 2.5, 4.0, 7.0, 10.0])
def test_dbn_matches_difference_of_library_root(gfo, n):
    h = 1e-4 * n
    fd = (sp.gammaincinv(2 * (n + h), 0.5) - sp.gammaincinv(2 * (n - h), 0.5)) / (2 * h)
    assert gfo.dbn(n) == pytest.approx(fd, rel=1e-7)


def test_dbn_asymptotic_slope(gfo):
    # Ciotti & Bertin (1999): b_n = 2n - 1/3 + 4/(405 n) + 46/(25515 n^2) + ...
    n = 10.0
    slope = 2.0 - 4.0 / (405 * n * n) - 92.0 / (25515 * n ** 3)
    assert gfo.dbn(n) == pytest.approx(slope, abs=1e-7)


# ----------------------------------------------------------- profile (D2) ---
@pytest.mark.parametrize("n,re,q,phi", [(0.5, 6.0, 0.7, 0.3), (1.0, 4.0, 0.4, 2.0), (2.5, 8.0, 0.7, math.pi / 6),
                                        (6.0, 3.0, 0.9, -1.1)])
def test_profile_along_axes(gfo, n, re, q, phi):
    """Along the major axis (cos phi, sin phi) the elliptical radius is the
    distance; along the minor axis it is distance / q; at R = Re the surface
    brightness is Ie; at the centre it is Ie e^{b_n}."""
    x0, y0, ie = 10.25, -3.5, 1.7
    c = [x0, y0, ie, re, n, q, phi]
    b = sp.gammaincinv(2 * n, 0.5)
    prof = lambda R: ie * math.exp(-b * ((R / re) ** (1.0 / n) - 1.0))
    for d in (0.3, re, 2.7 * re):
        xm, ym = x0 + d * math.cos(phi), y0 + d * math.sin(phi)
        assert gfo.sersic_point(c, xm, ym) == pytest.approx(prof(d), rel=1e-12)
        xn, yn = x0 - d * math.sin(phi), y0 + d * math.cos(phi)
        assert gfo.sersic_point(c, xn, yn) == pytest.approx(prof(d / q), rel=1e-12)
    assert gfo.sersic_point(c, x0 + re * math.cos(phi), y0 + re * math.sin(phi)) == pytest.approx(ie, rel=1e-12)
    assert gfo.sersic_point(c, x0, y0) == pytest.approx(ie * math.exp(b), rel=1e-13)


def _subsample_points(H, W, K, S):
    """Sub-sample centres of every padded pixel: x = j + (s+1/2)/S - 1/2."""
    c = (K - 1) // 2
    offs = (np.arange(S) + 0.5) / S - 0.5
    jj = np.arange(-c, W + c)
    ii = np.arange(-c, H + c)
    X = jj[None, :, None, None] + offs[None, None, None, :]
    Y = ii[:, None, None, None] + offs[None, None, :, None]
    return np.broadcast_arrays(X, Y)


def test_n_half_is_elliptical_gaussian(gfo):
    """n = 0.5 is a Gaussian with covariance Rot diag(s^2, (q s)^2) Rot^T,
    s^2 = Re^2 / (2 ln 2), peak 2 Ie.  Sampled at the same sub-sample centres."""
    H, W, K, S = 20, 17, 5, 5
    x0, y0, ie, re, q, phi = 8.3, 9.1, 1.3, 4.0, 0.55, 0.7
    th = np.array([x0, y0, ie, re, 0.5, q, phi, 0.0])
    img = gfo.eval_padded(H, W, K, th, S)
    s2 = re * re / (2 * math.log(2.0))
    rot = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
    cov = rot @ np.diag([s2, q * q * s2]) @ rot.T
    icov = np.linalg.inv(cov)
    X, Y = _subsample_points(H, W, K, S)
    dx, dy = X - x0, Y - y0
    qf = icov[0, 0] * dx * dx + 2 * icov[0, 1] * dx * dy + icov[1, 1] * dy * dy
    ref = (2 * ie * np.exp(-0.5 * qf)).mean(axis=(2, 3))
    np.testing.assert_allclose(img, ref, rtol=1e-12, atol=1e-300)


def test_n_one_is_exponential(gfo):
    """n = 1 is an exponential disk: Ie e^{b_1} exp(-b_1 R / Re)."""
    H, W, K, S = 16, 16, 3, 5
    x0, y0, ie, re, q, phi = 7.8, 8.15, 0.9, 3.0, 0.35, 2.4
    th = np.array([x0, y0, ie, re, 1.0, q, phi, 0.0])
    img = gfo.eval_padded(H, W, K, th, S)
    b1 = sp.gammaincinv(2.0, 0.5)
    major = np.array([math.cos(phi), math.sin(phi)])
    minor = np.array([-math.sin(phi), math.cos(phi)])
    X, Y = _subsample_points(H, W, K, S)
    dx, dy = X - x0, Y - y0
    R = np.hypot(dx * major[0] + dy * major[1], (dx * minor[0] + dy * minor[1]) / q)
    ref = (ie * math.exp(b1) * np.exp(-b1 * R / re)).mean(axis=(2, 3))
    np.testing.assert_allclose(img, ref, rtol=1e-12)


def _flux(n, re, q, ie):
    b = sp.gammaincinv(2 * n, 0.5)
    return 2 * math.pi * n * re * re * q * ie * math.exp(b) * b ** (-2 * n) * sp.gamma(2 * n)


@pytest.mark.parametrize("n,re,q,S,tol", [(0.5, 6.0, 0.6, 5, 1e-12), (1.0, 6.0, 0.6, 15, 2e-7),
                                          (1.5, 8.0, 0.6, 5, 2e-5), (2.0, 8.0, 0.6, 15, 1e-3)])
def test_total_flux_closed_form(gfo, n, re, q, S, tol):
    """Sum of pixels (unit area) equals 2 pi n Re^2 q Ie e^{b_n} b_n^{-2n} Gamma(2n)
    up to the midpoint-rule error of the sub-sampling (the flux outside the
    200x200 grid is below 1e-9 for these profiles)."""
    th = np.array([100.3, 99.6, 1.0, re, n, q, 0.4, 0.0])
    s = gfo.eval_padded(200, 200, 1, th, S).sum()
    assert s / _flux(n, re, q, 1.0) == pytest.approx(1.0, abs=tol)


@pytest.mark.parametrize("n,re,q", [(4.0, 10.0, 0.6), (6.0, 12.0, 0.6), (4.0, 4.0, 0.8)])
def test_flux_bracket_for_extended_profiles(gfo, n, re, q):
    """When the profile extends past the grid, the grid holds between
    F P(2n, b (R_in/Re)^{1/n}) and F P(2n, b (R_out/Re)^{1/n}) with R_in / R_out
    the elliptical radii of the largest inscribed / smallest enclosing ellipse."""
    x0, y0 = 100.3, 99.6
    th = np.array([x0, y0, 1.0, re, n, q, 0.4, 0.0])
    s = gfo.eval_padded(200, 200, 1, th, 15).sum() / _flux(n, re, q, 1.0)
    b = sp.gammaincinv(2 * n, 0.5)
    dmin = min(x0 + 0.5, 199.5 - x0, y0 + 0.5, 199.5 - y0)
    dmax = max(math.hypot(a, c) for a in (x0 + 0.5, 199.5 - x0) for c in (y0 + 0.5, 199.5 - y0))
    pin = sp.gammainc(2 * n, b * (dmin / re) ** (1 / n))
    pout = sp.gammainc(2 * n, b * (dmax / q / re) ** (1 / n))
    assert pin - 1e-3 <= s <= pout + 1e-3
    # and the bracket is tight enough to reject a wrong b_n (e.g. the 2n - 1/3 approximation used as exact)
    assert pout - pin < 0.07


def test_padding_geometry(gfo):
    """The padded grid starts at stamp pixel (-c, -c): its pixel (c, c) is stamp
    pixel (0, 0)."""
    th = np.array([3.2, 5.9, 1.0, 2.0, 1.3, 0.8, 0.2, 0.0])
    K = 7
    c = 3
    img = gfo.eval_padded(10, 12, K, th, 5)
    assert img.shape == (16, 18)
    for (i, j) in [(0, 0), (-3, -3), (9, 11), (12, 14), (4, 7)]:
        assert img[i + c, j + c] == gfo.pixel(th, 5, i, j)


# ----------------------------------------------------------- convolution (D6) ---
@pytest.mark.parametrize("K", [1, 3, 5, 7])
def test_conv_matches_scipy_valid(gfo, K):
    g = synth.rng(7 + K)
    mp = g.standard_normal((8 + K - 1, 11 + K - 1))
    psf = synth.random_psf(K, 100 + K)
    np.testing.assert_allclose(gfo.conv_valid(mp, psf), scipy.signal.convolve2d(mp, psf, mode="valid"),
                               rtol=1e-12, atol=1e-12)


def test_conv_brute_force_8x8(gfo):
    """Quadruple loop over output and taps with the flip written as index
    reversal of the kernel."""
    g = synth.rng(3)
    K = 5
    mp = g.standard_normal((8 + K - 1, 8 + K - 1))
    psf = synth.random_psf(K, 11)
    flipped = psf[::-1, ::-1]
    ref = np.zeros((8, 8))
    for y in range(8):
        for x in range(8):
            ref[y, x] = np.sum(flipped * mp[y:y + K, x:x + K])
    np.testing.assert_allclose(gfo.conv_valid(mp, psf), ref, rtol=1e-13, atol=1e-13)


def test_conv_matches_fft_product(gfo):
    """Linear convolution via the discrete Fourier transform of zero-padded
    operands (numpy.fft), cropped to the valid region."""
    g = synth.rng(5)
    K, Mh, Mw = 9, 30, 25
    mp = g.standard_normal((Mh, Mw))
    psf = synth.random_psf(K, 12)
    Fh, Fw = Mh + K - 1, Mw + K - 1
    full = np.fft.irfft2(np.fft.rfft2(mp, (Fh, Fw)) * np.fft.rfft2(psf, (Fh, Fw)), (Fh, Fw))
    np.testing.assert_allclose(gfo.conv_valid(mp, psf), full[K - 1:Mh, K - 1:Mw], atol=1e-12)


def test_delta_psf_is_identity(gfo):
    K = 9
    psf = np.zeros((K, K))
    psf[K // 2, K // 2] = 1.0
    th = np.array([11.2, 9.7, 1.0, 3.0, 2.2, 0.6, 0.9, 0.05])
    H, W = 21, 19
    mp = gfo.eval_padded(H, W, K, th, 5)
    out = gfo.conv_valid(mp, psf)
    c = K // 2
    np.testing.assert_array_equal(out, mp[c:c + H, c:c + W])
    m = gfo.model(H, W, th, psf, 5)
    np.testing.assert_allclose(m, mp[c:c + H, c:c + W] + 0.05, rtol=1e-15)


def test_gaussian_convolved_with_gaussian(gfo):
    """An n = 0.5 component convolved with a Gaussian PSF is the Gaussian with
    the summed covariance (same sub-sample averaging, same total flux).  The
    residual is PSF truncation at K = 21 for sigma_p = 1.5 (~1e-10) and
    aliasing of the pixel-sampled PSF (~exp(-2 pi^2 sigma_p^2))."""
    H = W = 40
    K, sp_ = 21, 1.5
    x0, y0, ie, re, q, phi = 19.6, 20.3, 1.0, 5.0, 0.5, 0.8
    th = np.array([x0, y0, ie, re, 0.5, q, phi, 0.0])
    psf = synth.gaussian_psf(K, sp_)
    m = gfo.model(H, W, th, psf, 5)
    s2 = re * re / (2 * math.log(2.0))
    rot = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
    cov1 = rot @ np.diag([s2, q * q * s2]) @ rot.T
    cov = cov1 + sp_ * sp_ * np.eye(2)
    amp = 2 * ie * math.sqrt(np.linalg.det(cov1) / np.linalg.det(cov))
    icov = np.linalg.inv(cov)
    X, Y = _subsample_points(H, W, 1, 5)
    dx, dy = X - x0, Y - y0
    ref = (amp * np.exp(-0.5 * (icov[0, 0] * dx * dx + 2 * icov[0, 1] * dx * dy + icov[1, 1] * dy * dy))).mean(
        axis=(2, 3))
    err = np.linalg.norm(m - ref) / np.linalg.norm(ref)
    assert err < 1e-6


# ------------------------------------------------------------------ chi^2 (D8) ---
def test_chi2_self_fit_is_zero_and_matches_sum(gfo):
    st = synth.c1()
    m = gfo.model(st.H, st.W, st.truth, st.psf, 5)
    w = np.full_like(m, 2500.0)
    assert gfo.chi2(m, w, m) == 0.0
    d, w = synth.add_gaussian_noise(m, 0.02, 5)
    c, r = gfo.chi2(d, w, m, want_resid=True)
    assert c == pytest.approx(math.fsum((w * (d - m) ** 2).ravel()), rel=1e-12)
    np.testing.assert_allclose(r, np.sqrt(w) * (d - m), rtol=1e-14)
    # masked pixels (w = 0) do not count
    w2 = w.copy()
    w2[:10] = 0
    assert gfo.chi2(d, w2, m) == pytest.approx(math.fsum((w2 * (d - m) ** 2).ravel()), rel=1e-12)


# ---------------------------------------------------------- derivatives (D9) ---
def _fd_jacobian(gfo, H, W, th, psf, S):
    P = th.size
    J = np.zeros((P, H, W))
    for p in range(P):
        h = 1e-6 * max(abs(th[p]), 1.0)
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        J[p] = (gfo.model(H, W, tp, psf, S) - gfo.model(H, W, tm, psf, S)) / (2 * h)
    return J


@pytest.mark.parametrize("th", [
    [8.3, 7.6, 1.2, 3.0, 2.5, 0.7, 0.5, 0.01],
    [8.45, 7.35, 0.8, 2.2, 0.7, 0.4, 2.1, 0.0],
    [7.9, 8.2, 1.0, 4.0, 4.3, 0.9, -0.4, 8.1, 8.05, 0.3, 6.0, 1.0, 0.5, 1.2, 0.1],
])
def test_jacobian_matches_central_differences(gfo, th):
    th = np.asarray(th, float)
    H = W = 16
    psf = synth.random_psf(5, 21)
    J = gfo.jacobian(H, W, th, psf, 5)
    Jfd = _fd_jacobian(gfo, H, W, th, psf, 5)
    for p in range(th.size):
        scale = np.abs(Jfd[p]).max()
        assert np.abs(J[p] - Jfd[p]).max() <= 2e-6 * scale + 1e-12, f"parameter {p}"


def test_grad_chi2_matches_central_differences(gfo):
    st = synth.c1()
    H, W = 24, 24
    th = np.array([11.7, 12.2, 1.0, 3.0, 2.0, 0.7, 0.5, 0.01])
    m = gfo.model(H, W, th, st.psf, 5)
    d, w = synth.add_gaussian_noise(m, 0.02, 9)
    th2 = th * np.array([1.01, 0.99, 1.05, 0.95, 1.03, 1.02, 0.9, 1.2])
    g = gfo.grad_chi2(th2, st.psf, d, w, 5)
    for p in range(th.size):
        h = 1e-6 * max(abs(th2[p]), 1.0)
        tp, tm = th2.copy(), th2.copy()
        tp[p] += h
        tm[p] -= h
        fd = (gfo.chi2(d, w, gfo.model(H, W, tp, st.psf, 5)) - gfo.chi2(d, w, gfo.model(H, W, tm, st.psf, 5))) / (
            2 * h)
        assert g[p] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(g).max())


# ------------------------------------------------------------------- LM (D11) ---
def test_lm_linear_parameters_match_lstsq(gfo):
    """With only Ie and sky free the model is linear in them; LM must land on
    the weighted least-squares solution from numpy.linalg.lstsq."""
    H = W = 24
    psf = synth.gaussian_psf(7, 1.2)
    th = np.array([11.7, 12.2, 1.0, 3.0, 2.0, 0.7, 0.5, 0.01])
    m = gfo.model(H, W, th, psf, 5)
    d, w = synth.add_gaussian_noise(m, 0.02, 13)
    template = gfo.model(H, W, np.r_[th[:2], 1.0, th[3:7], 0.0], psf, 5)
    A = np.stack([template.ravel(), np.ones(H * W)], 1) * np.sqrt(w.ravel())[:, None]
    sol = np.linalg.lstsq(A, d.ravel() * np.sqrt(w.ravel()), rcond=None)[0]
    free = np.zeros(8, np.uint8)
    free[[2, 7]] = 1
    start = th.copy()
    start[2], start[7] = 0.6, 0.03
    fit, info = gfo.fit_lm(start, psf, d, w, 5, free=free, ftol=1e-14, xtol=1e-14, max_iter=50)
    assert fit[2] == pytest.approx(sol[0], rel=1e-9)
    assert fit[7] == pytest.approx(sol[1], rel=1e-7, abs=1e-10)
    np.testing.assert_array_equal(fit[[0, 1, 3, 4, 5, 6]], th[[0, 1, 3, 4, 5, 6]])


def test_lm_truth_start_noise_free_stops_at_once(gfo):
    H = W = 20
    psf = synth.gaussian_psf(7, 1.2)
    th = np.array([9.7, 10.2, 1.0, 3.0, 2.0, 0.7, 0.5, 0.01])
    m = gfo.model(H, W, th, psf, 5)
    fit, info = gfo.fit_lm(th, psf, m, np.ones_like(m), 5)
    assert info["chi2"] == 0.0 and info["iters"] == 0 and info["status"] == 0 and info["reason"] == 3
    np.testing.assert_array_equal(fit, th)


def test_lm_recovers_truth_noise_free(gfo):
    H = W = 32
    psf = synth.gaussian_psf(9, 1.5)
    th = np.array([15.7, 16.2, 1.0, 4.0, 2.0, 0.7, 0.5, 0.01])
    m = gfo.model(H, W, th, psf, 5)
    start = synth.perturb_uniform(th, synth.rng(77), 0.2)
    lo, hi = synth.bounds(1, H, W)
    fit, info = gfo.fit_lm(start, psf, m, np.full_like(m, 2500.0), 5, lo=lo, hi=hi, ftol=1e-15, xtol=1e-13,
                           max_iter=200)
    np.testing.assert_allclose(fit, th, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("ncomp", [1, 2])
def test_lm_fit_on_noisy_data_is_a_stationary_point(gfo, ncomp):
    """The whole fit on noisy data has no closed form, but its end point has
    a property that needs no LM: chi^2 is stationary there.  At the oracle's
    fit (ftol 1e-13, every parameter inside its bounds) the central-difference
    gradient of the oracle's chi^2 along each parameter is tiny: a Newton
    step along that axis (gradient over second difference) would lower chi^2
    by less than 1e-9 of it, and chi^2 rises on both sides of the fit along
    every axis.  A wrong sign or a dropped factor in any Jacobian column, or a
    damping that stops short, leaves a gradient many orders above that."""
    H = W = 32
    psf = synth.gaussian_psf(9, 1.5)
    if ncomp == 1:
        th = np.array([15.7, 16.2, 1.0, 4.0, 2.0, 0.7, 0.5, 0.01])
    else:
        th = np.array([15.7, 16.2, 2.0, 2.5, 3.0, 0.8, 0.4, 15.6, 16.1, 0.5, 7.0, 1.0, 0.5, 1.2, 0.01])
    m = gfo.model(H, W, th, psf, 5)
    d, w = synth.add_gaussian_noise(m, 0.02, 91 + ncomp)
    start = synth.perturb_uniform(th, synth.rng(78 + ncomp), 0.1)
    lo, hi = synth.bounds(ncomp, H, W)
    fit, info = gfo.fit_lm(start, psf, d, w, 5, lo=lo, hi=hi, ftol=1e-13, xtol=1e-14, max_iter=300)
    # away from every finite bound (the open ones are +-1e30)
    margin = np.where(hi - lo < 1e20, 1e-3 * (hi - lo), 0.0)
    assert np.all(fit > lo + margin) and np.all(fit < hi - margin), fit

    def chi2(t):
        return gfo.chi2(d, w, gfo.model(H, W, t, psf, 5))

    c0 = chi2(fit)
    assert c0 == pytest.approx(info["chi2"], rel=1e-12)
    for p in range(fit.size):
        scale = max(abs(fit[p]), 1.0)
        h1, h2 = 1e-6 * scale, 1e-3 * scale
        e = np.zeros_like(fit)
        e[p] = 1.0
        g = (chi2(fit + h1 * e) - chi2(fit - h1 * e)) / (2 * h1)
        up, dn = chi2(fit + h2 * e), chi2(fit - h2 * e)
        curv = (up - 2 * c0 + dn) / h2 ** 2
        assert curv > 0 and up > c0 and dn > c0, (p, up - c0, dn - c0)
        assert g * g / (2 * curv) <= 1e-9 * c0, (p, g, curv, c0)


def test_lm_bounds_are_respected(gfo):
    H = W = 20
    psf = synth.gaussian_psf(7, 1.2)
    th = np.array([9.7, 10.2, 1.0, 3.0, 2.0, 0.95, 0.5, 0.01])
    m = gfo.model(H, W, th, psf, 5)
    d, w = synth.add_gaussian_noise(m, 0.02, 3)
    lo, hi = synth.bounds(1, H, W)
    hi[5] = 0.9  # force q against its upper bound
    fit, info = gfo.fit_lm(np.r_[th[:5], 0.8, th[6:]], psf, d, w, 5, lo=lo, hi=hi, max_iter=60)
    assert fit[5] <= 0.9
    assert np.all(fit >= lo) and np.all(fit <= hi)


# ------------------------------------------------ LM step and damping trace
def _fd_jacobian(gfo, H, W, th, psf, S=5):
    """Central differences of the oracle's model (independent of its
    analytic Jacobian)."""
    J = np.empty((th.size, H, W))
    for p in range(th.size):
        h = 1e-5 * max(abs(th[p]), 1.0)
        a, b = th.copy(), th.copy()
        a[p] += h
        b[p] -= h
        J[p] = (gfo.model(H, W, a, psf, S) - gfo.model(H, W, b, psf, S)) / (2 * h)
    return J


def _damped_step(J, w, r, lam, keep):
    """Marquardt's step on the parameters in keep: (A + lam D) delta = g with
    A = J^T W J, g = J^T W r, D = diag(max(A_ii, 1e-12 max_j A_jj)), by a
    general solve (not a Cholesky factorisation)."""
    Jk = J[keep].reshape(len(keep), -1)
    A = (Jk * w.ravel()) @ Jk.T
    g = (Jk * w.ravel()) @ r.ravel()
    D = np.maximum(np.diag(A), 1e-12 * np.diag(A).max())
    return np.linalg.solve(A + lam * np.diag(D), g)


def test_lm_damping_trace_across_rejections(gfo):
    """From a start far from the minimum the first four damped steps raise
    chi^2 and are rejected (lambda 1e-3 -> 1e-2 -> 0.1 -> 1 -> 10, the
    Jacobian kept), the fifth (lambda = 10) lowers it and is accepted
    (lambda -> 1).  Each trial point is recomputed here from a
    finite-difference Jacobian and a general linear solve; the oracle's
    state after k iterations must follow it."""
    H = W = 24
    psf = synth.gaussian_psf(5, 1.2)
    truth = np.array([12.3, 11.6, 1.0, 3.0, 2.5, 0.7, 0.5, 0.01])
    d, w = synth.add_gaussian_noise(gfo.model(H, W, truth, psf, 5), 0.02, 11)
    t0 = truth * np.array([1, 1, 0.3, 0.4, 3.0, 1, 1, 1])
    m0 = gfo.model(H, W, t0, psf, 5)
    c0 = float(np.sum(w * (d - m0) ** 2))
    J = _fd_jacobian(gfo, H, W, t0, psf)
    keep = list(range(8))
    lam, accepted_at = 1e-3, None
    for k in range(1, 6):
        trial = t0 + _damped_step(J, w, d - m0, lam, keep)
        ct = float(np.sum(w * (d - gfo.model(H, W, trial, psf, 5)) ** 2))
        th, info = gfo.fit_lm(t0, psf, d, w, 5, max_iter=k)
        assert info["njev"] == 1 and info["nfev"] == k + 1 and info["iters"] == k
        if ct < c0:
            accepted_at = k
            np.testing.assert_allclose(th, trial, rtol=1e-6, atol=1e-8)
            assert info["chi2"] == pytest.approx(ct, rel=1e-7)
            assert info["lam"] == pytest.approx(lam / 10.0, rel=1e-15)
            break
        np.testing.assert_array_equal(th, t0)      # rejected: theta stays
        assert info["chi2"] == pytest.approx(c0, rel=1e-12)
        lam *= 10.0
        assert info["lam"] == pytest.approx(lam, rel=1e-15)
    assert accepted_at == 5
    # the damping changes the step: the undamped (Gauss-Newton) step and a
    # unit-matrix damping both land far from the accepted point
    gn = t0 + _damped_step(J, w, d - m0, 0.0, keep)
    assert np.abs(gn - th).max() > 1e-2
    Jk = J.reshape(8, -1)
    A = (Jk * w.ravel()) @ Jk.T
    g = (Jk * w.ravel()) @ (d - m0).ravel()
    unit = t0 + np.linalg.solve(A + 10.0 * np.eye(8), g)
    assert np.abs(unit - th).max() > 1e-2


def test_lm_damping_floor_keeps_a_flat_direction_solvable(gfo):
    """A round component (q = 1) does not depend on phi, so phi's Jacobian
    column and its diagonal of A are exactly zero.  The floor
    1e-12 max_j A_jj in D keeps A + lambda D positive definite: the step is
    taken, phi does not move, and the other parameters take the step of the
    system without phi."""
    H = W = 24
    psf = synth.gaussian_psf(5, 1.2)
    truth = np.array([12.3, 11.6, 1.0, 3.0, 2.5, 1.0, 0.5, 0.01])
    d, w = synth.add_gaussian_noise(gfo.model(H, W, truth, psf, 5), 0.02, 12)
    t0 = truth * np.array([1.01, 0.99, 1.1, 1.1, 0.95, 1.0, 1.0, 1.2])
    J = _fd_jacobian(gfo, H, W, t0, psf)
    ref = gfo.jacobian(H, W, t0, psf, 5)
    assert np.all(ref[6] == 0.0)
    keep = [0, 1, 2, 3, 4, 5, 7]
    trial = t0.copy()
    trial[keep] += _damped_step(J, w, d - gfo.model(H, W, t0, psf, 5), 1e-3, keep)
    th, info = gfo.fit_lm(t0, psf, d, w, 5, max_iter=1)
    assert info["nfev"] == 2 and info["lam"] == pytest.approx(1e-4)
    assert th[6] == t0[6]
    np.testing.assert_allclose(th, trial, rtol=1e-6, atol=1e-8)
