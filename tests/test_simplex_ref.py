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


# ---------------------------------------------------------------------------
# One iteration of each branch, with the points worked out by hand from the
# rules (coefficients 1, 2, 1/2, 1/2) on the simplex (0,0), (1,0), (0,1)
# (x0 = (0,0), steps 1): the reference must evaluate exactly these points,
# in this order.

def _points(fun, max_iter=1):
    pts = []

    def f(x):
        pts.append(tuple(float(v) for v in x))
        return fun(x)

    NM.minimize(f, np.zeros(2), np.ones(2), ftol=0.0, max_iter=max_iter)
    return pts


START = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)]


def test_nm_expansion_kept():
    # f = (x-3)^2 + (y-3)^2: 18, 13, 13.  best (1,0) (first of the ties),
    # worst (0,0); centroid (1/2, 1/2); reflection (1,1): 8 < 13 -> expansion
    # (3/2, 3/2): 4.5 < 8, kept.
    pts = _points(lambda x: (x[0] - 3) ** 2 + (x[1] - 3) ** 2)
    assert pts == START + [(1.0, 1.0), (1.5, 1.5)]
    # the next iteration works on (3/2,3/2), (1,0), (0,1): worst (0,1) (13,
    # the higher index of the tie), centroid (5/4, 3/4), reflection (5/2, 1/2)
    assert _points(lambda x: (x[0] - 3) ** 2 + (x[1] - 3) ** 2, 2)[5] == (2.5, 0.5)


def test_nm_expansion_rejected_reflection_kept():
    # f = (x-1)^2 + (y-1)^2: 2, 1, 1; reflection (1,1): 0 < 1 -> expansion
    # (3/2,3/2): 0.5 >= 0, so the reflection is kept; the next iteration's
    # worst is (0,1) (1, the higher index), centroid (1, 1/2), reflection (2, 0)
    f = lambda x: (x[0] - 1) ** 2 + (x[1] - 1) ** 2
    assert _points(f) == START + [(1.0, 1.0), (1.5, 1.5)]
    assert _points(f, 2)[5] == (2.0, 0.0)


def test_nm_reflection_kept_and_worst_tie_to_higher_index():
    # f = (x+y-0.4)^2: 0.16, 0.36, 0.36.  The worst is (0,1), the higher index
    # of the tie; centroid (1/2, 0); reflection (1,-1): 0.16, not below the
    # best (0.16) but below the second worst (0.36): kept.  (With the tie
    # to the lower index the reflection would be (-1, 1).)
    assert _points(lambda x: (x[0] + x[1] - 0.4) ** 2) == START + [(1.0, -1.0)]


def test_nm_outside_contraction_kept():
    # g(s), s = x + y, piecewise linear through (0,10), (1,1), (1.5,0.5), (2,5):
    # vertices 10, 1, 1; reflection (1,1): 5, between the second worst (1)
    # and the worst (10) -> outside contraction (3/4, 3/4): 0.5 <= 5, kept.
    g = lambda x: float(np.interp(x[0] + x[1], [0, 1, 1.5, 2], [10, 1, 0.5, 5]))
    assert _points(g) == START + [(1.0, 1.0), (0.75, 0.75)]


def test_nm_outside_contraction_rejected_then_shrink():
    # as above with g(1.5) = 7: the contraction (3/4, 3/4) gives 7 > 5 = f_r,
    # so it is not kept (the rule compares with the reflection, not with
    # the worst, 10) and every vertex but the best (1,0) moves halfway to
    # it: (1/2, 0), then (1/2, 1/2).
    g = lambda x: float(np.interp(x[0] + x[1], [0, 1, 1.5, 2], [10, 1, 7, 5]))
    assert _points(g) == START + [(1.0, 1.0), (0.75, 0.75), (0.5, 0.0), (0.5, 0.5)]


def test_nm_inside_contraction_kept():
    # f = x^2 + 10 y^2: 0, 1, 10; worst (0,1), centroid (1/2, 0); reflection
    # (1,-1): 11 >= 10 -> inside contraction (1/4, 1/2): 2.5625 < 10, kept.
    assert _points(lambda x: x[0] ** 2 + 10 * x[1] ** 2) == START + [(1.0, -1.0), (0.25, 0.5)]


def test_nm_inside_contraction_rejected_then_shrink():
    # f = x + 2|y| + 10 exp(-((x - 1/4)^2 + (y - 1/2)^2)/0.01): about 0, 1, 2;
    # reflection (1,-1): 3 >= 2 -> inside contraction (1/4, 1/2): 11.25 >= 2,
    # not kept -> shrink towards the best (0,0): (1/2, 0), (0, 1/2).
    f = lambda x: x[0] + 2 * abs(x[1]) + 10 * np.exp(-((x[0] - 0.25) ** 2 + (x[1] - 0.5) ** 2) / 0.01)
    assert _points(f) == START + [(1.0, -1.0), (0.25, 0.5), (0.5, 0.0), (0.0, 0.5)]
