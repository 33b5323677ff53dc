"""Seeded synthetic inputs for the galaxy-fitting workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
holds none of the fitting method's arithmetic: it draws parameter vectors,
PSF images, noise fields and batch size lists from numpy ``PCG64`` streams, and
turns a noise-free model image (rendered by whichever implementation the
caller uses) into an observation with noise and inverse-variance weights.

Parameter vectors are ``[x0, y0, Ie, Re, n, q, phi] * ncomp + [sky]`` with
``phi`` in radians (counter-clockwise from +x, x along columns) and the
pixel (row i, col j) centred on (x=j, y=i).

Workloads (image shapes and parameter ranges follow the survey-cutout-like
configurations the build is measured on; they are synthetic stand-ins, the
paper measures on no public dataset):
  C1  one 64x64 stamp, one Sersic component, 15x15 Gaussian PSF, 8 parameters
  C2  one 512x512 image, bulge + exponential disk, 65x65 Moffat PSF, 15 parameters
  C3  4096 stamps of uneven size, per-stamp Gaussian or Moffat PSF (15..33 px)
  C4  1024 perturbed parameter vectors against one 256x256 image, 33x33 Moffat
  C5  128x128 training / evaluation stamps drawn with the C3 priors
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1000
C3_SIZES = (32, 48, 64, 96, 128, 192, 256)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ------------------------------------------------------------------ PSF images
def gaussian_psf(K: int, sigma: float) -> np.ndarray:
    """K x K circular Gaussian sampled at pixel centres (centre index (K-1)/2),
    normalised to unit sum in FP64.  Returned as float64."""
    if K % 2 == 0:
        raise ValueError("PSF side must be odd")
    c = (K - 1) / 2
    y, x = np.mgrid[0:K, 0:K].astype(np.float64)
    r2 = (x - c) ** 2 + (y - c) ** 2
    p = np.exp(-r2 / (2.0 * sigma * sigma))
    return p / p.sum()


def moffat_alpha(fwhm: float, beta: float) -> float:
    return fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))


def moffat_psf(K: int, fwhm: float, beta: float = 3.0) -> np.ndarray:
    """K x K Moffat (1 + r^2/alpha^2)^-beta, alpha from the FWHM, unit sum."""
    if K % 2 == 0:
        raise ValueError("PSF side must be odd")
    a = moffat_alpha(fwhm, beta)
    c = (K - 1) / 2
    y, x = np.mgrid[0:K, 0:K].astype(np.float64)
    r2 = (x - c) ** 2 + (y - c) ** 2
    p = (1.0 + r2 / (a * a)) ** (-beta)
    return p / p.sum()


def random_psf(K: int, seed: int) -> np.ndarray:
    """Asymmetric random non-negative K x K kernel (unit sum) for convolution
    tests: a flip or transpose error changes the result."""
    g = rng(seed)
    p = g.random((K, K)) + np.linspace(0.0, 1.0, K)[None, :] * 2.0 + np.linspace(0.0, 3.0, K)[:, None]
    return p / p.sum()


# ---------------------------------------------------------------- observations
def add_gaussian_noise(model_true: np.ndarray, sigma: float, seed: int):
    """d = m + sigma z with z ~ N(0, 1); w = 1/sigma^2 everywhere."""
    z = rng(seed).standard_normal(model_true.shape)
    d = model_true + sigma * z
    w = np.full(model_true.shape, 1.0 / (sigma * sigma))
    return d, w


def add_poisson_read_noise(model_true: np.ndarray, read_noise: float, gain: float, seed: int):
    """Poisson (gain e-/ADU) plus Gaussian read noise, Gaussian-approximated:
    var = read^2 + max(m, 0)/gain; d = m + sqrt(var) z; w = 1/var."""
    var = read_noise * read_noise + np.maximum(model_true, 0.0) / gain
    z = rng(seed).standard_normal(model_true.shape)
    return model_true + np.sqrt(var) * z, 1.0 / var


# ------------------------------------------------------------------ workloads
@dataclass
class Stamp:
    H: int
    W: int
    psf: np.ndarray          # K x K float64, unit sum
    truth: np.ndarray        # P float64
    start: np.ndarray        # P float64 (perturbed initial guess)
    noise_sigma: float = 0.02
    noise_seed: int = 0
    kind: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return self.psf.shape[0]

    @property
    def ncomp(self) -> int:
        return (self.truth.size - 1) // 7


def bounds(ncomp: int, H: int, W: int):
    """Box bounds clipped after every LM step: n in [0.2, 10], q in [0.05, 1],
    Re >= 0.1, Ie >= 1e-6, centre within +-N/2 of the stamp centre."""
    lo, hi = [], []
    for _ in range(ncomp):
        lo += [W / 2 - W / 2, H / 2 - H / 2, 1e-6, 0.1, 0.2, 0.05, -1e30]
        hi += [W / 2 + W / 2, H / 2 + H / 2, 1e30, 1e30, 10.0, 1.0, 1e30]
    lo.append(-1e30)
    hi.append(1e30)
    return np.array(lo), np.array(hi)


def perturb_uniform(truth: np.ndarray, g: np.random.Generator, frac: float = 0.2) -> np.ndarray:
    """theta (1 + u), u ~ U[-frac, frac] per parameter; each centre coordinate
    moves by u * Re of its component instead."""
    t = truth.copy()
    nc = (t.size - 1) // 7
    for k in range(nc):
        re = truth[7 * k + 3]
        for p in range(7):
            u = g.uniform(-frac, frac)
            if p in (0, 1):
                t[7 * k + p] = truth[7 * k + p] + u * re
            else:
                t[7 * k + p] = truth[7 * k + p] * (1.0 + u)
    t[-1] = truth[-1] * (1.0 + g.uniform(-frac, frac))
    return t


def c1(seed: int = SEED_BASE + 1) -> Stamp:
    """Single 64x64 stamp: n=2.5, Re=8, q=0.7, PA=30 deg, Ie=1, centre
    (32.3, 31.7), sky 0.01, 15x15 Gaussian PSF sigma=1.5, noise sigma=0.02,
    start perturbed by +-20%."""
    g = rng(seed)
    truth = np.array([32.3, 31.7, 1.0, 8.0, 2.5, 0.7, math.pi / 6, 0.01])
    start = perturb_uniform(truth, g, 0.2)
    return Stamp(64, 64, gaussian_psf(15, 1.5), truth, start, 0.02, seed * 10 + 7, "C1")


def c2(seed: int = SEED_BASE + 2) -> Stamp:
    """512x512 bulge + exponential disk on a sky of 100 e-, 65x65 Moffat PSF
    (beta=3, FWHM=3), Poisson (gain 1) + read noise 5 e-, 15 free parameters.
    Bulge n~U[2,6], Re~U[5,20], q~U[0.6,1], Ie=100; disk n=1, Re~U[20,60],
    q~U[0.3,1], Ie=20; shared centre 256 + U[-1,1]; PAs ~U[0, pi].
    Start: +-10% on every parameter, centre moved by +-0.1 Re_bulge."""
    g = rng(seed)
    cx, cy = 256 + g.uniform(-1, 1), 256 + g.uniform(-1, 1)
    bulge = [cx, cy, 100.0, g.uniform(5, 20), g.uniform(2, 6), g.uniform(0.6, 1.0), g.uniform(0, math.pi)]
    disk = [cx, cy, 20.0, g.uniform(20, 60), 1.0, g.uniform(0.3, 1.0), g.uniform(0, math.pi)]
    truth = np.array(bulge + disk + [100.0])
    start = truth.copy()
    for p in range(15):
        u = g.uniform(-0.1, 0.1)
        if p in (0, 1, 7, 8):
            start[p] = truth[p] + u * truth[3]
        else:
            start[p] = truth[p] * (1.0 + u)
    return Stamp(512, 512, moffat_psf(65, 3.0, 3.0), truth, start, 0.0, seed * 10 + 7, "C2",
                 meta=dict(read_noise=5.0, gain=1.0))


def c3_stamp(g: np.random.Generator, N: int, idx: int, seed: int) -> Stamp:
    n = g.uniform(0.5, 6.0)
    re = g.uniform(2.0, 0.25 * N)
    q = g.uniform(0.2, 1.0)
    pa = g.uniform(0.0, math.pi)
    ie = math.exp(g.uniform(math.log(0.5), math.log(5.0)))
    cx, cy = N / 2 + g.uniform(-1, 1), N / 2 + g.uniform(-1, 1)
    sky = g.uniform(0.0, 0.05)
    K = int(g.choice(np.arange(15, 34, 2)))
    fwhm = g.uniform(2.0, 4.0)
    if g.random() < 0.5:
        psf = gaussian_psf(K, fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0))))
        kind = "gauss"
    else:
        psf = moffat_psf(K, fwhm, 3.0)
        kind = "moffat"
    truth = np.array([cx, cy, ie, re, n, q, pa, sky])
    start = perturb_uniform(truth, g, 0.2)
    return Stamp(N, N, psf, truth, start, 0.02, seed * 100000 + idx, "C3:" + kind)


def c3_psf(g: np.random.Generator) -> np.ndarray:
    """PSF from the uneven-batch distribution: K odd ~ U{15..33}, FWHM ~ U[2, 4],
    Gaussian or Moffat (beta 3) with probability 1/2."""
    K = int(g.choice(np.arange(15, 34, 2)))
    fwhm = g.uniform(2.0, 4.0)
    if g.random() < 0.5:
        return gaussian_psf(K, fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0))))
    return moffat_psf(K, fwhm, 3.0)


def psf_bank(n: int, seed: int):
    """n PSFs drawn with c3_psf (training seed 2000, evaluation seed 3000)."""
    g = rng(seed)
    return [c3_psf(g) for _ in range(n)]


def c3(n_stamps: int = 4096, seed: int = SEED_BASE + 3, sizes=C3_SIZES):
    """Batch of uneven single-Sersic stamps: side ~ U{32,...,256}, n~U[0.5,6],
    Re~U[2, N/4], q~U[0.2,1], PA~U[0,pi], Ie log-uniform [0.5,5], centre
    N/2 + U[-1,1], sky U[0,0.05], noise 0.02; per-stamp Gaussian or Moffat
    (beta=3) PSF with K odd in 15..33 and FWHM~U[2,4]."""
    g = rng(seed)
    out = []
    for i in range(n_stamps):
        N = int(g.choice(np.asarray(sizes)))
        out.append(c3_stamp(g, N, i, seed))
    return out


def c4_truth():
    """256x256 image: n=2.5, Re=24, q=0.7, PA=30 deg, Ie=1, centre
    (128.3, 127.7), sky 0.01, noise 0.02, 33x33 Moffat PSF (beta=3, FWHM=3)."""
    truth = np.array([128.3, 127.7, 1.0, 24.0, 2.5, 0.7, math.pi / 6, 0.01])
    return Stamp(256, 256, moffat_psf(33, 3.0, 3.0), truth, truth.copy(), 0.02, (SEED_BASE + 4) * 10 + 7, "C4")


def c4_vectors(step: int, n_vec: int = 1024) -> np.ndarray:
    """Parameter vectors of one likelihood step: theta_i (1 + 0.05 z), the
    centre moved by 0.05 Re z and the PA by 0.05 pi z, z ~ N(0,1).  Step s
    draws from seed 1004*10^4 + s."""
    truth = c4_truth().truth
    g = rng((SEED_BASE + 4) * 10000 + step)
    z = g.standard_normal((n_vec, truth.size))
    th = np.repeat(truth[None, :], n_vec, axis=0)
    th[:, 0] += 0.05 * truth[3] * z[:, 0]
    th[:, 1] += 0.05 * truth[3] * z[:, 1]
    for p in (2, 3, 4, 5, 7):
        th[:, p] = truth[p] * (1.0 + 0.05 * z[:, p])
    th[:, 6] = truth[6] + 0.05 * math.pi * z[:, 6]
    th[:, 5] = np.clip(th[:, 5], 0.05, 1.0)
    return th


# ------------------------------------------------------------ spectral lines
# Spectra for the 1-D line-fitting family: N channels, 1..3 Gaussian emission
# lines [A, mu, sigma] (peak, centre and width in channels) plus a constant
# continuum, a K-tap Gaussian line-spread function.  Shaped like integral-
# field or long-slit spectra around a few emission lines.
LINE_SIZES = (256, 512, 1024, 2048)


def gaussian_lsf(K: int, sigma: float) -> np.ndarray:
    """K taps of a Gaussian sampled at integer offsets from the centre tap,
    unit sum (float64)."""
    if K % 2 == 0:
        raise ValueError("LSF length must be odd")
    x = np.arange(K, dtype=np.float64) - (K - 1) / 2
    v = np.exp(-x * x / (2.0 * sigma * sigma))
    return v / v.sum()


@dataclass
class Spectrum:
    N: int
    lsf: np.ndarray
    truth: np.ndarray
    start: np.ndarray
    noise_sigma: float
    noise_seed: int

    @property
    def K(self) -> int:
        return int(self.lsf.size)

    @property
    def nlines(self) -> int:
        return (self.truth.size - 1) // 3


def line_spectrum(g: np.random.Generator, N: int, nlines: int, idx: int, seed: int) -> Spectrum:
    """Lines with A ~ log-U[0.5, 5], mu ~ U[0.15 N, 0.85 N], sigma ~ U[1.5, 6];
    continuum ~ U[0, 0.5]; LSF K ~ U{7, 9, ..., 21}, sigma_lsf ~ U[0.8, 2.5];
    noise sigma 0.05.  Start: A and sigma x (1 + U[-0.2, 0.2]), mu + U[-0.5, 0.5]
    sigma, continuum + U[-0.05, 0.05]."""
    t, s = [], []
    for _ in range(nlines):
        a = math.exp(g.uniform(math.log(0.5), math.log(5.0)))
        mu = g.uniform(0.15 * N, 0.85 * N)
        sg = g.uniform(1.5, 6.0)
        t += [a, mu, sg]
        s += [a * (1.0 + g.uniform(-0.2, 0.2)), mu + g.uniform(-0.5, 0.5) * sg, sg * (1.0 + g.uniform(-0.2, 0.2))]
    cont = g.uniform(0.0, 0.5)
    t.append(cont)
    s.append(cont + g.uniform(-0.05, 0.05))
    K = int(g.choice(np.arange(7, 22, 2)))
    lsf = gaussian_lsf(K, g.uniform(0.8, 2.5))
    return Spectrum(N, lsf, np.array(t), np.array(s), 0.05, seed * 100003 + idx)


def line_batch(n: int, seed: int = SEED_BASE + 6, sizes=LINE_SIZES):
    g = rng(seed)
    return [line_spectrum(g, int(g.choice(sizes)), int(g.integers(1, 4)), i, seed) for i in range(n)]


def line_bounds(nlines: int, N: int):
    """A in [0, 1e30], mu in [0, N - 1], sigma in [0.3, N / 4], continuum free."""
    lo, hi = [], []
    for _ in range(nlines):
        lo += [0.0, 0.0, 0.3]
        hi += [1e30, N - 1.0, N / 4.0]
    lo.append(-1e30)
    hi.append(1e30)
    return np.array(lo), np.array(hi)


def add_noise_1d(model_true: np.ndarray, sigma: float, seed: int):
    """Observation and inverse-variance weights for a 1-D model."""
    g = rng(seed)
    d = model_true + sigma * g.standard_normal(model_true.shape)
    w = np.full(model_true.shape, 1.0 / (sigma * sigma))
    return d, w


# ------------------------------------------------------------------ data cubes
CUBE_SIZES = (32, 40, 48, 56, 64)


@dataclass
class Cube:
    H: int
    W: int
    Nc: int
    psf: np.ndarray
    lsf: np.ndarray
    truth: np.ndarray
    start: np.ndarray
    noise_sigma: float
    noise_seed: int

    @property
    def K(self) -> int:
        return int(self.psf.shape[0])

    @property
    def Kl(self) -> int:
        return int(self.lsf.size)


def cube_stamp(g: np.random.Generator, H: int, W: int, Nc: int, lsf: np.ndarray, idx: int, seed: int) -> Cube:
    """An integral-field cube of a rotating disk galaxy, parameters
    [xc, yc, Ie, Re, n, q, phi, continuum, v0, vproj, rt, sigma_v]:
    centre (W/2, H/2) + U[-1, 1], Ie log-U[0.5, 5], Re ~ U[2, max(min(H, W)/5, 2.5)],
    n ~ U[0.6, 2.5], q ~ U[0.35, 0.95], phi ~ U[0, pi], continuum U[0, 0.05],
    v0 ~ Nc/2 + U[-2, 2], vproj ~ U[2, max(Nc/6, 2.5)], rt ~ U[1, 0.8 Re],
    sigma_v ~ U[1.2, 3] channels; Gaussian or Moffat PSF with K in
    {9, 11, 13, 15} and FWHM ~ U[2, 3.5]; noise sigma 0.02.  Start: the
    profile parameters x (1 + U[-0.1, 0.1]) (the centre moves by U[-0.1, 0.1] Re),
    v0 + U[-1, 1], vproj, rt and sigma_v x (1 + U[-0.15, 0.15]), continuum
    + U[-0.01, 0.01]."""
    re = g.uniform(2.0, max(min(H, W) / 5.0, 2.5))
    t = np.array([W / 2 + g.uniform(-1, 1), H / 2 + g.uniform(-1, 1), math.exp(g.uniform(math.log(0.5), math.log(5.0))),
                  re, g.uniform(0.6, 2.5), g.uniform(0.35, 0.95), g.uniform(0.0, math.pi), g.uniform(0.0, 0.05),
                  Nc / 2 + g.uniform(-2, 2), g.uniform(2.0, max(Nc / 6.0, 2.5)), g.uniform(1.0, 0.8 * re), g.uniform(1.2, 3.0)])
    K = int(g.choice([9, 11, 13, 15]))
    fwhm = g.uniform(2.0, 3.5)
    psf = gaussian_psf(K, fwhm / 2.3548200450309493) if g.uniform() < 0.5 else moffat_psf(K, fwhm, 3.0)
    s = t.copy()
    for p in range(7):
        u = g.uniform(-0.1, 0.1)
        s[p] = t[p] + u * re if p < 2 else t[p] * (1.0 + u)
    s[7] = t[7] + g.uniform(-0.01, 0.01)
    s[8] = t[8] + g.uniform(-1, 1)
    for p in (9, 10, 11):
        s[p] = t[p] * (1.0 + g.uniform(-0.15, 0.15))
    return Cube(H, W, Nc, psf, lsf, t, s, 0.02, seed * 100019 + idx)


def cube_batch(n: int, seed: int = SEED_BASE + 7, sizes=CUBE_SIZES, Nc: int = 64, Kl: int = 7,
               sigma_lsf: float = 1.1):
    """n cubes of N x N spaxels, N ~ U{sizes}, Nc channels, one Gaussian LSF of
    Kl taps for the batch."""
    g = rng(seed)
    lsf = gaussian_lsf(Kl, sigma_lsf)
    out = []
    for i in range(n):
        N = int(g.choice(sizes))
        out.append(cube_stamp(g, N, N, Nc, lsf, i, seed))
    return out


def cube_bounds(H: int, W: int, Nc: int):
    """Box bounds of a cube's parameters: the profile's as ``bounds(1, H, W)``,
    continuum free, v0 in [0, Nc - 1], vproj free, rt >= 0.1,
    sigma_v in [0.3, Nc / 4]."""
    lo, hi = bounds(1, H, W)
    lo = np.r_[lo, 0.0, -1e30, 0.1, 0.3]
    hi = np.r_[hi, Nc - 1.0, 1e30, 1e30, Nc / 4.0]
    return lo, hi
