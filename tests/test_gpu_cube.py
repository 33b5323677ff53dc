"""GPU parity of the data-cube path (gf_cube_*) against the FP64 cube oracle
(oracle/cube_ref.py), through the C ABI:

* model cubes of a ragged batch (direct, one-workgroup FFT and multi-pass
  FFT spatial convolutions; several oversampling factors): relative L2
  <= 1e-5 per cube;
* chi^2 within 1e-5 chi^2 plus the FP32 model-error term
  2 eps sqrt(chi^2) ||sqrt(w) m|| (eps = 2e-6);
* Jacobian cubes: relative L2 <= 1e-4 per parameter, the continuum's all ones;
* LM fits of a batch at the parameter-parity tolerance (ftol 1e-12):
  parameters within 1e-4 max(|theta|, s), chi^2 within 1e-5 of the oracle's
  fit on the same FP32 observation;
* a cube fitted alone gives the same bits as inside the batch;
* argument errors."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cube_ref as CR
from paper_1101_2254_amd import ops
from paper_1101_2254_amd import _lib as L
from tests.gpu_common import rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("gpu cube: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _cubes(shapes, Nc, Kl, seed):
    """Cubes of the given (H, W, K) with the synthetic priors."""
    g = synth.rng(seed)
    lsf = synth.gaussian_lsf(Kl, 1.1)
    out = []
    for i, (H, W, K) in enumerate(shapes):
        c = synth.cube_stamp(g, H, W, Nc, lsf, i, seed)
        c.psf = synth.gaussian_psf(K, 1.2) if K > 1 else np.ones((1, 1))
        out.append(c)
    return out


class GpuCubes:
    def __init__(self, ctx, cubes, thetas=None, mode=ops.GF_CONV_AUTO, data=None, weights=None):
        self.cubes = cubes
        Nc, Kl = cubes[0].Nc, cubes[0].Kl
        self.cb = ops.CubeBatch(ctx, [c.H for c in cubes], [c.W for c in cubes], [c.K for c in cubes], Nc, Kl)
        self.psf32 = [c.psf.astype(np.float32) for c in cubes]
        self.lsf32 = [c.lsf.astype(np.float32) for c in cubes]
        self.cb.set_kernels(to_dev(np.concatenate([p.ravel() for p in self.psf32])),
                            to_dev(np.concatenate(self.lsf32)), mode)
        thetas = thetas if thetas is not None else [c.truth for c in cubes]
        self.th = [np.asarray(t, np.float64) for t in thetas]
        self.theta = to_dev(np.concatenate(self.th), torch.float64)
        if data is not None:
            self.d32 = [np.asarray(x, np.float32) for x in data]
            self.w32 = [np.asarray(x, np.float32) for x in weights]
            self.data = to_dev(np.concatenate([x.ravel() for x in self.d32]))
            self.weight = to_dev(np.concatenate([x.ravel() for x in self.w32]))

    def split(self, flat, per=1):
        f = flat.detach().cpu().numpy()
        out = []
        for s, c in enumerate(self.cubes):
            o = int(self.cb.offsets["vox"][s]) * per
            n = c.Nc * c.H * c.W
            out.append(f[o:o + per * n].reshape((per, c.Nc, c.H, c.W) if per > 1 else (c.Nc, c.H, c.W)))
        return out

    def oracle_model(self, s, S, Sv, theta=None):
        c = self.cubes[s]
        return CR.model(self.th[s] if theta is None else theta, c.H, c.W, self.psf32[s].astype(np.float64),
                        self.lsf32[s].astype(np.float64), c.Nc, S, Sv)


SHAPES = [(20, 24, 5), (33, 27, 9), (16, 16, 1), (40, 36, 15)]


@pytest.mark.parametrize("S,Sv,mode", [(3, 2, ops.GF_CONV_AUTO), (5, 3, ops.GF_CONV_AUTO),
                                       (2, 1, L.GF_CONV_FFT_MULTIPASS), (1, 4, L.GF_CONV_FFT_FUSED)])
def test_cube_model_ragged_batch(ctx, S, Sv, mode):
    shapes = SHAPES if mode == ops.GF_CONV_AUTO else [s for s in SHAPES if s[2] > 1]
    cubes = _cubes(shapes, 18, 5, 500 + S)
    gc = GpuCubes(ctx, cubes, mode=mode)
    print(f"cube model S={S} Sv={Sv} mode={mode}", flush=True)
    m = gc.split(ops.cube_model(gc.cb.ctx, gc.cb, gc.theta, S, Sv))
    for s in range(len(cubes)):
        ref = gc.oracle_model(s, S, Sv)
        assert rel_l2(m[s], ref) <= 1e-5, (s, rel_l2(m[s], ref))


def test_cube_model_edge_parameters(ctx):
    """Cusp and flattening extremes: n = 6, q = 0.1, centre on a spaxel (a
    sub-sample at R = 0), a fast narrow line near the band edge."""
    cubes = _cubes([(24, 24, 7), (21, 19, 3)], 16, 3, 77)
    th0 = cubes[0].truth.copy()
    th0[[0, 1, 4, 5]] = [12.0, 12.0, 6.0, 0.1]
    th1 = cubes[1].truth.copy()
    th1[[8, 9, 10, 11]] = [2.5, 7.0, 0.5, 0.6]
    gc = GpuCubes(ctx, cubes, thetas=[th0, th1])
    m = gc.split(ops.cube_model(ctx, gc.cb, gc.theta, 3, 3))
    for s in range(2):
        ref = gc.oracle_model(s, 3, 3)
        assert rel_l2(m[s], ref) <= 1e-5, (s, rel_l2(m[s], ref))


def test_cube_chi2(ctx):
    cubes = _cubes(SHAPES[:3], 18, 5, 600)
    data, w = [], []
    for i, c in enumerate(cubes):
        m = CR.model(c.truth, c.H, c.W, c.psf, c.lsf, c.Nc, 3, 2)
        d, ww = synth.add_gaussian_noise(m, 0.02, 900 + i)
        data.append(d)
        w.append(ww)
    gc = GpuCubes(ctx, cubes, thetas=[c.start for c in cubes], data=data, weights=w)
    c2 = ops.cube_chi2(ctx, gc.cb, gc.theta, gc.data, gc.weight, 3, 2).cpu().numpy().astype(np.float64)
    for s in range(len(cubes)):
        mo = gc.oracle_model(s, 3, 2)
        dd, ww = gc.d32[s].astype(np.float64), gc.w32[s].astype(np.float64)
        ref = CR.chi2(dd, ww, mo)
        got = c2[s, 0] + c2[s, 1]
        bound = 1e-5 * ref + 2 * 2e-6 * math.sqrt(ref) * np.linalg.norm(np.sqrt(ww) * mo)
        assert abs(got - ref) <= bound, (s, got, ref, bound)


def test_cube_jacobian(ctx):
    cubes = _cubes([(18, 20, 5), (22, 22, 9)], 14, 5, 700)
    gc = GpuCubes(ctx, cubes, thetas=[c.start for c in cubes])
    print("cube jacobian", flush=True)
    J = gc.split(ops.cube_jacobian(ctx, gc.cb, gc.theta, 3, 2), per=CR.NPAR)
    for s, c in enumerate(cubes):
        ref = CR.jacobian(gc.th[s], c.H, c.W, gc.psf32[s].astype(np.float64), gc.lsf32[s].astype(np.float64), c.Nc,
                          3, 2)
        for p in range(CR.NPAR):
            assert rel_l2(J[s][p], ref[p]) <= 1e-4, (s, p, rel_l2(J[s][p], ref[p]))
        assert np.all(J[s][CR.CONT] == 1.0)


def _observe(cubes, S, Sv, seed):
    data, weights = [], []
    for i, c in enumerate(cubes):
        m = CR.model(c.truth, c.H, c.W, c.psf.astype(np.float32).astype(np.float64),
                     c.lsf.astype(np.float32).astype(np.float64), c.Nc, S, Sv)
        d, w = synth.add_gaussian_noise(m, c.noise_sigma, seed + i)
        data.append(d)
        weights.append(w)
    return data, weights


def _bounds(cubes):
    lo = np.concatenate([synth.cube_bounds(c.H, c.W, c.Nc)[0] for c in cubes])
    hi = np.concatenate([synth.cube_bounds(c.H, c.W, c.Nc)[1] for c in cubes])
    return lo, hi


FIT = dict(ftol=1e-12, xtol=1e-10, max_iter=200)


@pytest.fixture(scope="module")
def cube_fit(ctx):
    cubes = _cubes([(20, 20, 5), (24, 22, 9), (18, 18, 7)], 14, 5, 800)
    data, w = _observe(cubes, 3, 2, 810)
    gc = GpuCubes(ctx, cubes, thetas=[c.start for c in cubes], data=data, weights=w)
    lo, hi = _bounds(cubes)
    print("cube LM fit of the batch", flush=True)
    fit, res = ops.cube_fit_lm(ctx, gc.cb, gc.data, gc.weight, gc.theta, 2, lo=to_dev(lo, torch.float64),
                               hi=to_dev(hi, torch.float64), oversample=3, **FIT)
    return cubes, gc, fit.cpu().numpy(), res, lo, hi


@pytest.mark.parametrize("s", [0, 1, 2])
def test_cube_fit_matches_oracle(cube_fit, s):
    cubes, gc, fit, res, lo, hi = cube_fit
    c = cubes[s]
    print(f"oracle fit of cube {s}", flush=True)
    ref, info = CR.fit_lm(c.start, gc.psf32[s].astype(np.float64), gc.lsf32[s].astype(np.float64),
                          gc.d32[s].astype(np.float64), gc.w32[s].astype(np.float64), 3, 2,
                          lo=lo[12 * s:12 * s + 12], hi=hi[12 * s:12 * s + 12], **FIT)
    # at ftol 1e-12 the FP32 chi^2 of the GPU fit stops improving before the
    # relative drop gets that small, so its fit ends on the step size or the
    # damping cap; the point it reaches is what is compared
    print(f"gpu: iters {res['iters'][s]} reason {res['reason'][s]}; oracle {info}", flush=True)
    assert res["chi2"][s] == pytest.approx(info["chi2"], rel=1e-5)
    a = fit[12 * s:12 * s + 12]
    re = abs(ref[CR.RE])
    for p in range(CR.NPAR):
        if p == CR.PHI:
            dphi = (a[p] - ref[p] + math.pi / 2) % math.pi - math.pi / 2
            assert abs(dphi) <= 1e-4 * math.pi, (p, a[p], ref[p])
            continue
        scale = re if p in (CR.XC, CR.YC) else c.noise_sigma if p == CR.CONT else 1.0 if p >= CR.V0 else 0.0
        assert abs(a[p] - ref[p]) <= 1e-4 * max(abs(ref[p]), scale), (p, a[p], ref[p])


def test_cube_fit_alone_same_bits(ctx, cube_fit):
    cubes, gc, fit, res, lo, hi = cube_fit
    s = 1
    one = GpuCubes(ctx, [cubes[s]], thetas=[cubes[s].start], data=[gc.d32[s]], weights=[gc.w32[s]])
    f1, r1 = ops.cube_fit_lm(ctx, one.cb, one.data, one.weight, one.theta, 2,
                             lo=to_dev(lo[12 * s:12 * s + 12], torch.float64),
                             hi=to_dev(hi[12 * s:12 * s + 12], torch.float64), oversample=3, **FIT)
    np.testing.assert_array_equal(f1.cpu().numpy(), fit[12 * s:12 * s + 12])
    assert r1["chi2"][0] == res["chi2"][s] and r1["iters"][0] == res["iters"][s]


def test_cube_errors(ctx):
    with pytest.raises(RuntimeError):
        ops.CubeBatch(ctx, [16], [16], [5], 0, 5)          # no channels
    with pytest.raises(RuntimeError):
        ops.CubeBatch(ctx, [16], [16], [5], 8, 4)          # even LSF
    with pytest.raises(RuntimeError):
        ops.CubeBatch(ctx, [16], [16], [4], 8, 5)          # even PSF
    cb = ops.CubeBatch(ctx, [16], [16], [5], 8, 5)
    theta = to_dev(np.zeros(12), torch.float64)
    with pytest.raises(RuntimeError):
        ops.cube_model(ctx, cb, theta)                     # kernels not set
    cb.set_kernels(to_dev(np.ones(25) / 25), to_dev(np.ones(5) / 5))
    with pytest.raises(RuntimeError):
        ops.cube_model(ctx, cb, theta, 9, 1)              # oversample out of range


def test_cube_fit_default_tolerance_converges(ctx, cube_fit):
    """At ftol 1e-5 every cube stops on the chi^2 rule, at a chi^2 within
    1e-4 of the minimum the tight fit reached."""
    cubes, gc, fit, res, lo, hi = cube_fit
    f2, r2 = ops.cube_fit_lm(ctx, gc.cb, gc.data, gc.weight, gc.theta, 2, lo=to_dev(lo, torch.float64),
                             hi=to_dev(hi, torch.float64), oversample=3, ftol=1e-5)
    assert np.all(r2["status"] == 0) and np.all(r2["reason"] == 1), r2
    for s in range(len(cubes)):
        assert res["chi2"][s] * (1 - 1e-6) <= r2["chi2"][s] <= res["chi2"][s] * (1 + 1e-4)


def test_cube_bench_configuration(ctx):
    """The benchmarked cube batch's launch configuration (its first cubes:
    32..64 spaxels, 64 channels, 9..15 px PSFs, 7-tap LSF, S = 5, Sv = 3):
    models of one cube per size against the oracle, the Jacobian of a 48 px
    cube, and a fit of a 32 px cube at the parameter-parity tolerance."""
    allc = synth.cube_batch(256)
    pick = []
    for N in synth.CUBE_SIZES:
        pick.append(next(i for i, c in enumerate(allc) if c.H == N))
    cubes = [allc[i] for i in pick]
    print("bench-configuration cubes", [(c.H, c.K) for c in cubes], flush=True)
    gc = GpuCubes(ctx, cubes, thetas=[c.start for c in cubes])
    m = gc.split(ops.cube_model(ctx, gc.cb, gc.theta, 5, 3))
    for s in range(len(cubes)):
        ref = gc.oracle_model(s, 5, 3)
        assert rel_l2(m[s], ref) <= 1e-5, (s, rel_l2(m[s], ref))
    s48 = [c.H for c in cubes].index(48)
    J = gc.split(ops.cube_jacobian(ctx, gc.cb, gc.theta, 5, 3), per=CR.NPAR)[s48]
    c = cubes[s48]
    ref = CR.jacobian(gc.th[s48], c.H, c.W, gc.psf32[s48].astype(np.float64), gc.lsf32[s48].astype(np.float64), c.Nc,
                      5, 3)
    for p in range(CR.NPAR):
        assert rel_l2(J[p], ref[p]) <= 1e-4, (p, rel_l2(J[p], ref[p]))
    # a fit of the 32 px cube inside the five-cube batch
    data, w = _observe(cubes, 5, 3, 4242)
    gd = GpuCubes(ctx, cubes, thetas=[c.start for c in cubes], data=data, weights=w)
    lo, hi = _bounds(cubes)
    fit, res = ops.cube_fit_lm(ctx, gd.cb, gd.data, gd.weight, gd.theta, 3, lo=to_dev(lo, torch.float64),
                               hi=to_dev(hi, torch.float64), oversample=5, **FIT)
    fit = fit.cpu().numpy()
    s = 0
    c = cubes[s]
    print("oracle fit of the 32 px cube", flush=True)
    ref, info = CR.fit_lm(c.start, gd.psf32[s].astype(np.float64), gd.lsf32[s].astype(np.float64),
                          gd.d32[s].astype(np.float64), gd.w32[s].astype(np.float64), 5, 3,
                          lo=lo[:12], hi=hi[:12], **FIT)
    assert res["chi2"][s] == pytest.approx(info["chi2"], rel=1e-5)
    a = fit[:12]
    for p in range(CR.NPAR):
        if p == CR.PHI:
            assert abs((a[p] - ref[p] + math.pi / 2) % math.pi - math.pi / 2) <= 1e-4 * math.pi
            continue
        scale = abs(ref[CR.RE]) if p in (CR.XC, CR.YC) else c.noise_sigma if p == CR.CONT else \
            1.0 if p >= CR.V0 else 0.0
        assert abs(a[p] - ref[p]) <= 1e-4 * max(abs(ref[p]), scale), (p, a[p], ref[p])


@pytest.mark.parametrize("shapes,Nc,Kl", [([(1, 1, 1), (2, 3, 3)], 1, 1), ([(3, 2, 1), (5, 4, 3)], 5, 3),
                                          ([(6, 6, 3)], 1024, 5)])
def test_cube_degenerate_and_maximum_shapes(ctx, shapes, Nc, Kl):
    """One spaxel, one channel, delta kernels, and the longest spectral axis."""
    cubes = _cubes(shapes, Nc, Kl, 31)
    th = []
    for c in cubes:
        t = c.truth.copy()
        t[[0, 1, 3]] = [c.W / 2 - 0.3, c.H / 2 + 0.2, 1.5]
        t[8] = Nc / 2 + 0.4
        th.append(t)
    gc = GpuCubes(ctx, cubes, thetas=th)
    m = gc.split(ops.cube_model(ctx, gc.cb, gc.theta, 3, 2))
    J = gc.split(ops.cube_jacobian(ctx, gc.cb, gc.theta, 3, 2), per=CR.NPAR)
    for s, c in enumerate(cubes):
        ref = gc.oracle_model(s, 3, 2)
        assert rel_l2(m[s], ref) <= 1e-5, (s, rel_l2(m[s], ref))
        if Nc <= 5:
            rj = CR.jacobian(gc.th[s], c.H, c.W, gc.psf32[s].astype(np.float64), gc.lsf32[s].astype(np.float64), Nc,
                             3, 2)
            for p in range(CR.NPAR):
                if np.linalg.norm(rj[p]) > 1e-12:
                    assert rel_l2(J[s][p], rj[p]) <= 1e-4, (s, p, rel_l2(J[s][p], rj[p]))
