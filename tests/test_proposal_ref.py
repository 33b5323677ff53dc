"""CPU pins of the references behind the starting-point path: Philox4x64-10
and its Gaussian draws, the parameter coding, the prior draw and the
image-moment default guess."""
import math

import numpy as np
import pytest

from oracle import cnn_ref as C
from oracle import moments_ref as MR
from oracle import philox_ref as PX
from oracle import gfo


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((0x1234, 0xABCDEF), (5, 0, 0, 0)),
                                     ((2000, 1), ((1 << 64) - 2, 7, 0, 3))])
def test_philox_matches_numpy(key, ctr):
    """numpy's Philox increments its counter before each block, so its first
    block is ours at counter + 1."""
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = g.random_raw(4 * 5)
    mine = PX.raw_blocks(key, PX.counter_add(ctr, 1), 5).reshape(-1)
    assert np.array_equal(raw, mine)


def test_counter_carry():
    assert PX.counter_add([(1 << 64) - 1, (1 << 64) - 1, 0, 0], 1) == [0, 0, 1, 0]


def test_box_muller_pairs_and_moments():
    key, ctr = (7, 9), (0, 0, 0, 0)
    z = PX.normals(key, ctr, 4 * 20000)
    w = PX.raw_blocks(key, ctr, 20000)
    u = PX.uniform24(w)
    # the pair (z0, z1) has squared radius -2 ln u0 and angle 2 pi u1
    r2 = z[0::4] ** 2 + z[1::4] ** 2
    np.testing.assert_allclose(r2, -2 * np.log(u[:, 0]), rtol=1e-12)
    ang = np.mod(np.arctan2(z[1::4], z[0::4]), 2 * np.pi)
    np.testing.assert_allclose(np.cos(ang), np.cos(2 * np.pi * u[:, 1]), atol=1e-9)
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1) < 0.02


def test_uniform24_range():
    w = np.array([0, (1 << 64) - 1], dtype=np.uint64)
    u = PX.uniform24(w)
    assert u[0] == 0.5 / (1 << 24) and u[1] == 1 - 0.5 / (1 << 24)


def test_coding_round_trip():
    g = np.random.default_rng(5)
    n, side = 200, 128
    th = np.stack([side / 2 + g.uniform(-1, 1, n), side / 2 + g.uniform(-1, 1, n), np.exp(g.uniform(-0.7, 1.6, n)),
                   g.uniform(2, 32, n), g.uniform(0.5, 6, n), g.uniform(0.2, 1, n), g.uniform(0, np.pi, n),
                   g.uniform(0, 0.05, n)], axis=1)
    back = C.decode(C.encode(th, side), side)
    np.testing.assert_allclose(back[:, [0, 1, 2, 3, 4, 5, 7]], th[:, [0, 1, 2, 3, 4, 5, 7]], rtol=1e-12, atol=1e-12)
    dphi = np.abs(np.mod(back[:, 6] - th[:, 6] + np.pi / 2, np.pi) - np.pi / 2)
    assert np.all(dphi[th[:, 5] < 0.999] < 1e-9)


def test_coding_box_edges_map_to_unit_interval():
    side = 128
    th = np.array([[64, 64, 0.5, 2, 0.5, 1.0, 0, 0], [64, 64, 5.0, 32, 6.0, 0.2, np.pi / 2, 0.05]])
    t = C.encode(th, side)
    np.testing.assert_allclose(t[:, 2:5], [[-1, -1, -1], [1, 1, 1]], atol=1e-12)
    np.testing.assert_allclose(t[:, 7], [-1, 1], atol=1e-12)
    np.testing.assert_allclose(t[1, 5:7], [-1, 0], atol=1e-12)   # (1 - q) cos(pi) / 0.8


def test_prior_draw_uses_the_stated_uniforms():
    key, ctr, n, side = (2000, 0x9A1A), (0, 0, 0, 0), 64, 128
    th = C.draw_prior(key, ctr, n, side)
    u = PX.uniform24(PX.raw_blocks(key, ctr, 2 * n)).reshape(n, 8)
    np.testing.assert_allclose(th[:, 4], 0.5 + 5.5 * u[:, 0])
    assert np.all((th[:, 3] >= 2) & (th[:, 3] <= side / 4))
    assert np.all((th[:, 5] >= 0.2) & (th[:, 5] <= 1) & (th[:, 2] >= 0.5) & (th[:, 2] <= 5))
    assert np.all(np.abs(th[:, :2] - side / 2) <= 1)


# ---------------------------------------------------------------- moments guess
def _frame_noise(H, W, sky, delta):
    """Frame of alternating sky +/- delta (median sky, RMS delta), sky inside."""
    d = np.full((H, W), sky)
    m = MR.frame_mask(H, W)
    idx = np.flatnonzero(m)
    d.flat[idx[0::2]] += delta
    d.flat[idx[1::2]] -= delta
    return d


def test_sky_is_the_frame_median_and_zero_weight_outside():
    d = _frame_noise(32, 32, 3.0, 0.1)
    th = MR.guess(d)
    assert th[7] == pytest.approx(3.0, abs=1e-15)
    assert th[3] == 2.0 and th[5] == 1.0   # no positive weight: fallback shape


def test_uniform_disk_half_light_radius():
    """v = A inside a disk of radius rho: C(r) grows as the disk area, so the
    half-weight radius is rho / sqrt(2) up to pixelisation."""
    H = W = 128
    rho = 40.0
    d = _frame_noise(H, W, 1.0, 0.01)
    yy, xx = np.mgrid[0:H, 0:W]
    disk = (xx - 64) ** 2 + (yy - 64) ** 2 <= rho ** 2
    d[disk] = 1.0 + 5.0
    th = MR.guess(d)
    assert th[0] == pytest.approx(64, abs=1e-9) and th[1] == pytest.approx(64, abs=1e-9)
    assert th[5] == pytest.approx(1.0, abs=2e-3)
    assert th[3] == pytest.approx(rho / math.sqrt(2), rel=1e-2)


@pytest.mark.parametrize("q,phi", [(0.5, 0.3), (0.7, 2.0), (0.35, math.pi / 2)])
def test_elliptical_gaussian_axes(q, phi):
    """An elliptical Gaussian (n = 0.5) of axis ratio q and angle phi: every
    isophote and every weight level is an ellipse of that shape, so the
    weighted second moments recover q and phi up to pixelisation."""
    H = W = 96
    yy, xx = np.mgrid[0:H, 0:W].astype(float)
    dx, dy = xx - 48, yy - 48
    xp = dx * math.cos(phi) + dy * math.sin(phi)
    yp = -dx * math.sin(phi) + dy * math.cos(phi)
    img = np.exp(-(xp ** 2 + (yp / q) ** 2) / (2 * 6.0 ** 2))
    d = _frame_noise(H, W, 0.0, 0.01) + img
    th = MR.guess(d)
    assert th[0] == pytest.approx(48, abs=1e-6) and th[1] == pytest.approx(48, abs=1e-6)
    assert th[5] == pytest.approx(q, rel=2e-2)
    dphi = abs((th[6] - phi + math.pi / 2) % math.pi - math.pi / 2)
    assert dphi < 1e-2


def test_flux_normalisation_matches_the_sersic_closed_form():
    """Ie is chosen so that the n = 2 closed-form total flux equals sum(d - sky)."""
    H = W = 64
    d = _frame_noise(H, W, 0.5, 0.01)
    yy, xx = np.mgrid[0:H, 0:W]
    d[(xx - 32) ** 2 + (yy - 30) ** 2 <= 100] += 2.0
    th = MR.guess(d)
    F = float(np.sum(d - th[7]))
    assert MR.sersic_total_flux(th[2], th[3], 2.0, th[5]) == pytest.approx(F, rel=1e-12)
    # the closed form against direct integration of q * 2 pi R I(R) dR
    from scipy.integrate import quad
    b = gfo.bn(2.0)
    num = quad(lambda r: 2 * math.pi * r * 0.6 * math.exp(-b * ((r / 3.0) ** 0.5 - 1)), 0, np.inf, limit=400)[0]
    assert MR.sersic_total_flux(1.0, 3.0, 2.0, 0.6) == pytest.approx(num, rel=1e-8)


# ---------------------------------------------------------------- multi-start
def test_multistart_reference_rules():
    from oracle import multistart_ref as MS
    th = np.array([[10.0, 11.0, 2.0, 5.0, 2.5, 0.6, 2.0, 0.01]])
    st = MS.expand_starts(th, 4)
    np.testing.assert_array_equal(st[0], th[0])
    assert st[1][4] == 1.0 and st[1][3] == 7.5 and st[2][4] == 4.0 and st[2][3] == pytest.approx(3.5)
    assert st[3][6] == pytest.approx(2.0 + math.pi / 2 - math.pi)
    np.testing.assert_array_equal(np.delete(st[3], 6), np.delete(th[0], 6))
    chi2 = np.array([5.0, 3.0, 3.0, np.nan, 1.0, 2.0])
    status = np.array([0, 0, 0, 0, 6, 6])
    assert list(MS.group_best([[0, 1, 2, 3], [4, 5]], chi2, status)) == [1, 4]
