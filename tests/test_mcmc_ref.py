"""CPU pins of the Metropolis reference: it samples a known Gaussian target,
respects the prior box, and a zero step always accepts without moving."""
import numpy as np
import pytest

from oracle import mcmc_ref as M


def test_gaussian_target_moments():
    """chi2 = sum ((theta - mu)/sigma)^2: the chain's stationary law is
    N(mu, sigma^2) per coordinate."""
    mu, sig = np.array([1.0, -2.0]), np.array([0.5, 2.0])
    f = lambda c, th: float(np.sum(((th - mu) / sig) ** 2))
    nc, n = 4, 3000
    th0 = np.tile(mu, (nc, 1))
    scale = np.tile(2.4 / np.sqrt(2) * sig, (nc, 1))
    st, ch, acc, _ = M.run(th0, scale, n, f, key=(11, 22))
    x = st[300:].reshape(-1, 2)
    assert np.all(np.abs(x.mean(0) - mu) < 0.15 * sig)
    assert np.all(np.abs(x.std(0) / sig - 1) < 0.12)
    assert 0.2 < acc.mean() < 0.6
    np.testing.assert_allclose(ch[-1], [f(0, s) for s in st[-1]])


def test_box_rejects_and_zero_step_accepts():
    f = lambda c, th: float(np.sum(th ** 2))
    th0 = np.array([[0.3, 0.4]])
    st, _, acc, margin = M.run(th0, np.array([[0.5, 0.5]]), 20, f, key=(1, 2), lo=th0, hi=th0)
    assert np.all(st == th0) and not acc.any() and np.all(np.isinf(margin))
    st, _, acc, _ = M.run(th0, np.zeros((1, 2)), 10, f, key=(1, 2))
    assert acc.all() and np.all(st == th0)


def test_continuation_is_the_same_chain():
    f = lambda c, th: float(np.sum(th ** 2))
    th0 = np.zeros((2, 3))
    sc = np.full((2, 3), 0.7)
    a, ca, _, _ = M.run(th0, sc, 10, f, key=(5, 6), stream=3)
    b1, _, _, _ = M.run(th0, sc, 4, f, key=(5, 6), stream=3)
    b2, cb, _, _ = M.run(b1[-1], sc, 6, f, key=(5, 6), stream=3, step0=4)
    np.testing.assert_array_equal(a, np.concatenate([b1, b2]))
