"""The benchmarked configurations at their full sizes against the FP64
oracle on oracle-rendered observations: the fit of one 512x512 image (Sersic
bulge + exponential disk, 65x65 Moffat PSF, 576-point FFT, 15 parameters, the
speculative iterations a single stamp takes by default), and the likelihood
step of 1024 parameter vectors against one 256x256 image (33x33 Moffat PSF,
288-point FFT) on sampled vectors."""
import math

import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import _lib as L
from paper_1101_2254_amd import ops
from tests.gpu_common import GpuBatch, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("gpu full size: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def test_c2_fit_full_size_matches_oracle(ctx, gfo):
    st = synth.c2()
    psf64 = st.psf.astype(np.float32).astype(np.float64)
    m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64), psf64, 5)
    d, w = synth.add_poisson_read_noise(m, st.meta["read_noise"], st.meta["gain"], st.noise_seed)
    gb = GpuBatch(ctx, [st], data=[d], weights=[w], mode=ops.GF_CONV_FFT)
    assert list(gb.psf.uses_fft) == [1] and list(gb.psf.fft_side) == [576]
    lo, hi = synth.bounds(2, st.H, st.W)
    d64, w64 = gb.d32[0].astype(np.float64), gb.w32[0].astype(np.float64)
    print("oracle fit of the 512x512 image", flush=True)
    ref, rinfo = gfo.fit_lm(st.start, psf64, d64, w64, 5, lo=lo, hi=hi, ftol=1e-8)
    assert rinfo["status"] == 0, rinfo
    for ftol in (1e-8, 1e-5):
        print(f"GPU fit, ftol {ftol}", flush=True)
        th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(st.start, torch.float64),
                              lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=ftol)
        th = th.cpu().numpy()
        assert info["status"][0] == L.GF_OK or info["reason"][0] == 4, info
        # the reported chi^2 is the oracle's at the returned parameters
        mt = gfo.model(st.H, st.W, th, psf64, 5)
        c_at = gfo.chi2(d64, w64, mt)
        wm = math.sqrt(float(np.sum(w64 * mt * mt)))
        assert abs(info["chi2"][0] - c_at) <= 1e-5 * c_at + 2 * 2e-6 * math.sqrt(c_at) * wm, (info["chi2"][0], c_at)
        # the same minimum: chi^2 within the tolerance the fit stops at
        assert info["chi2"][0] == pytest.approx(rinfo["chi2"], rel=max(ftol, 1e-6)), (info["chi2"][0], rinfo)
        if ftol == 1e-8:
            for k in range(2):
                re = abs(ref[7 * k + 3])
                for p in range(7):
                    i = 7 * k + p
                    if p == 6:
                        dd = (th[i] - ref[i] + math.pi / 2) % math.pi - math.pi / 2
                        assert abs(dd) <= 1e-4 * math.pi, (i, th[i], ref[i])
                    else:
                        s = re if p in (0, 1) else 0.0
                        assert abs(th[i] - ref[i]) <= 1e-4 * max(abs(ref[i]), s), (i, th[i], ref[i])
            assert abs(th[-1] - ref[-1]) <= 1e-4 * abs(ref[-1]), (th[-1], ref[-1])


def test_c4_likelihood_full_batch_sampled(ctx, gfo):
    base = synth.c4_truth()
    psf64 = base.psf.astype(np.float32).astype(np.float64)
    m = gfo.model(256, 256, base.truth.astype(np.float32).astype(np.float64), psf64, 5)
    d, w = synth.add_gaussian_noise(m, 0.02, base.noise_seed)
    th = synth.c4_vectors(0, 1024)
    gb = GpuBatch(ctx, [base] * 1024, thetas=list(th), data=[d], weights=[w], shared=True)
    assert list(gb.psf.fft_side)[:1] == [288]
    print("likelihood of 1024 vectors", flush=True)
    chi = ops.pairs_to_f64(ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5)).cpu().numpy()
    assert np.all(np.isfinite(chi))
    d64, w64 = gb.d32[0].astype(np.float64), gb.w32[0].astype(np.float64)
    for s in (0, 1, 255, 511, 777, 1023):
        mt = gfo.model(256, 256, gb.th64(s), psf64, 5)
        ref = gfo.chi2(d64, w64, mt)
        # away from the minimum the FP32 model error enters through the cross
        # term (Cauchy-Schwarz), as in the other trial-point checks
        wm = math.sqrt(float(np.sum(w64 * mt * mt)))
        assert abs(chi[s] - ref) <= 1e-5 * ref + 2 * 2e-6 * math.sqrt(ref) * wm, (s, chi[s], ref)


def test_c3_full_batch_sampled(gfo):
    """The uneven batch at its full size and in the benchmark's launch
    configuration: 4096 stamps of 32..256 px in one gf_fit_lm call at ftol
    1e-5 with at most 100 iterations, the count read after every iteration,
    two lanes, one-workgroup stamps moving to the multi-pass launches once few
    of their size remain.  The first stamp of each side gets an observation
    rendered by the oracle (the others one rendered by the library), and its
    final chi^2 is within 1e-5 (relative) of the oracle's fit from the same
    start."""
    ctx = ops.Context(0)
    stamps = synth.c3(4096)
    n = len(stamps)
    batch = ops.Batch(ctx, [s.H for s in stamps], [s.W for s in stamps], [s.K for s in stamps], [1] * n)
    taps = to_dev(np.concatenate([s.psf.ravel() for s in stamps]), torch.float32)
    psf = ops.Psf(ctx, batch, taps, ops.GF_CONV_AUTO)
    truth = to_dev(np.concatenate([s.truth for s in stamps]), torch.float32)
    print("library render of 4096 stamps", flush=True)
    m = ops.model(ctx, batch, psf, truth, 5).cpu().numpy().astype(np.float64)
    pick = {}
    for i, s in enumerate(stamps):
        pick.setdefault(s.H, i)
    assert sorted(pick) == sorted(synth.C3_SIZES)
    assert {1, 2} <= set(int(psf.uses_fft[i]) for i in pick.values())
    off = batch.offsets["pix"]
    d, w = np.empty_like(m), np.empty_like(m)
    for i, s in enumerate(stamps):
        sl = slice(off[i], off[i] + s.H * s.W)
        mi = m[sl].reshape(s.H, s.W)
        if i in pick.values():
            print(f"oracle render of stamp {i} ({s.H} px, K = {s.K})", flush=True)
            mi = gfo.model(s.H, s.W, s.truth.astype(np.float32).astype(np.float64),
                           s.psf.astype(np.float32).astype(np.float64), 5)
        dd, ww = synth.add_gaussian_noise(mi, s.noise_sigma, s.noise_seed)
        d[sl], w[sl] = dd.ravel(), ww.ravel()
    d32, w32 = d.astype(np.float32), w.astype(np.float32)
    lo = np.concatenate([synth.bounds(1, s.H, s.W)[0] for s in stamps])
    hi = np.concatenate([synth.bounds(1, s.H, s.W)[1] for s in stamps])
    start = np.concatenate([s.start for s in stamps])
    print("fit of 4096 stamps", flush=True)
    _, res = ops.fit_lm(ctx, batch, psf, to_dev(d32), to_dev(w32), to_dev(start, torch.float64),
                        lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=1e-5, max_iter=100,
                        poll_every=1)
    assert np.all(res["iters"] >= 1)
    for N, i in sorted(pick.items()):
        s = stamps[i]
        sl = slice(off[i], off[i] + s.H * s.W)
        l, h = synth.bounds(1, s.H, s.W)
        print(f"oracle fit of stamp {i} ({N} px)", flush=True)
        _, info = gfo.fit_lm(s.start, s.psf.astype(np.float32).astype(np.float64),
                             d32[sl].reshape(s.H, s.W).astype(np.float64), w32[sl].reshape(s.H, s.W).astype(np.float64),
                             5, lo=l, hi=h, ftol=1e-5, max_iter=100)
        assert info["status"] == 0, (i, N, info)
        assert res["status"][i] == 0 or res["reason"][i] == 4, (i, N, res[i])
        assert res["chi2"][i] == pytest.approx(info["chi2"], rel=1e-5), (i, N, res[i], info)
    torch.cuda.synchronize()
    ctx.close()
