"""CPU pins of the Nelder-Mead reference: known minima of textbook test
functions, the prior box, and the bookkeeping of its trace."""
import numpy as np
import pytest

from oracle import simplex_ref as NM


def test_quadratic_minimum():
    A = np.array([[3.0, 0.5, 0.0], [0.5, 2.0, 0.3], [0.0, 0.3, 1.0]])
    xs = np.array([1.0, -2.0, 0.5])
    f = lambda x: float((x - xs) @ A @ (x - xs)) + 4.0
    x, fb, it, nfev, ok, trace, _ = NM.minimize(f, np.zeros(3), np.full(3, 0.5), ftol=1e-14, max_iter=5000)
    assert ok and fb == pytest.approx(4.0, abs=1e-12)
    np.testing.assert_allclose(x, xs, atol=1e-5)
    assert nfev == len(trace) and min(trace) == fb


def test_rosenbrock():
    f = lambda x: 100.0 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
    x, fb, *_ = NM.minimize(f, np.array([-1.2, 1.0]), np.array([0.1, 0.1]), ftol=1e-16, max_iter=5000)
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-4)


def test_box_is_respected():
    f = lambda x: float(np.sum((x - 3.0) ** 2))
    lo, hi = np.array([-1.0, -1.0]), np.array([1.0, 2.0])
    x, fb, *_ = NM.minimize(f, np.zeros(2), np.array([0.3, 0.3]), lo=lo, hi=hi, ftol=1e-14)
    np.testing.assert_allclose(x, [1.0, 2.0], atol=1e-6)
