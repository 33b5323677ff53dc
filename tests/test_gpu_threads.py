"""Contexts used from several host threads at once: each thread fits its own
batch in its own context (graph capture, replay and the restriction of the
work lists to the stamps still iterating all happen while the other threads
capture and replay theirs), and every fit gives the bits that the same fit
gives when it runs alone."""
import threading

import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import ops
from tests.gpu_common import GpuBatch, to_dev

pytestmark = pytest.mark.gpu


def _problem(ctx, gfo, seed):
    g = synth.rng(seed)
    stamps = [synth.c3_stamp(g, int(N), i, seed * 10 + i) for i, N in enumerate([32, 48, 64, 96, 32, 128, 48, 64])]
    data, weights = [], []
    for s in stamps:
        m = gfo.model(s.H, s.W, s.truth.astype(np.float32).astype(np.float64),
                      s.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, s.noise_seed)
        data.append(d)
        weights.append(w)
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    lo = to_dev(np.concatenate([synth.bounds(1, s.H, s.W)[0] for s in stamps]), torch.float64)
    hi = to_dev(np.concatenate([synth.bounds(1, s.H, s.W)[1] for s in stamps]), torch.float64)
    start = to_dev(np.concatenate([s.start for s in stamps]), torch.float64)

    def fit():
        th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-8,
                              poll_every=1)
        return th.cpu().numpy(), info

    return fit, gb


def test_contexts_in_concurrent_threads(gfo):
    n = 3
    ctxs = [ops.Context(0) for _ in range(n)]
    streams = [torch.cuda.Stream() for _ in range(n)]
    probs = []
    for k in range(n):
        with torch.cuda.stream(streams[k]):
            probs.append(_problem(ctxs[k], gfo, 600 + k))
    torch.cuda.synchronize()
    print("fits one after another", flush=True)
    ref = []
    for k in range(n):
        with torch.cuda.stream(streams[k]):
            ref.append(probs[k][0]())
    torch.cuda.synchronize()
    out = [None] * n
    errs = []

    def run(k):
        try:
            with torch.cuda.stream(streams[k]):
                for _ in range(2):   # a replay of the kept graph, then another
                    out[k] = probs[k][0]()
        except Exception as e:   # reported below, in the main thread
            errs.append(f"{k}: {e}")

    print("fits in concurrent threads", flush=True)
    th = [threading.Thread(target=run, args=(k,)) for k in range(n)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in th)
    torch.cuda.synchronize()
    assert not errs, errs
    for k in range(n):
        np.testing.assert_array_equal(out[k][0], ref[k][0], err_msg=str(k))
        for f in ("chi2", "iters", "nfev", "njev", "status"):
            np.testing.assert_array_equal(out[k][1][f], ref[k][1][f], err_msg=f"{k} {f}")
    for c in ctxs:
        c.close()


def _lane_fitter(gfo):
    """600 stamps of 32 and 48 px (every seventh with a 5 px PSF, on the
    direct path), observed through the oracle, and a function fitting any
    subset of them in one call of a context that keeps the FFT forms."""
    from tests.gpu_common import keep_fft_forms
    ctx = ops.Context(0)
    keep_fft_forms(ctx)
    g = synth.rng(777)
    stamps = [synth.c3_stamp(g, int(g.choice([32, 48])), i, 777) for i in range(600)]
    for i in range(0, 600, 7):
        stamps[i].psf = synth.gaussian_psf(5, 1.0)   # direct-path stamps too
    data, weights = [], []
    for s in stamps:
        m = gfo.model(s.H, s.W, s.truth.astype(np.float32).astype(np.float64),
                      s.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, s.noise_seed)
        data.append(d)
        weights.append(w)

    def fit(idx, **kw):
        sts = [stamps[i] for i in idx]
        gb = GpuBatch(ctx, sts, data=[data[i] for i in idx], weights=[weights[i] for i in idx])
        lo = to_dev(np.concatenate([synth.bounds(1, s.H, s.W)[0] for s in sts]), torch.float64)
        hi = to_dev(np.concatenate([synth.bounds(1, s.H, s.W)[1] for s in sts]), torch.float64)
        start = to_dev(np.concatenate([s.start for s in sts]), torch.float64)
        th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-5, **kw)
        return th.cpu().numpy(), info, gb.batch.offsets["par"]

    return ctx, fit


def _same_stamps(one, two, lo_, hi_):
    t1, i1, p1 = one
    t2, i2, p2 = two
    for k, s in enumerate(range(lo_, hi_)):
        np.testing.assert_array_equal(t1[p1[k]:p1[k] + 8], t2[p2[s]:p2[s] + 8], err_msg=str(s))
        for f in ("chi2", "iters", "nfev", "njev", "status"):
            assert i1[f][k] == i2[f][s], (s, f, i1[f][k], i2[f][s])


def test_two_lanes_match_one_lane(gfo):
    """A plain-form batch of at least 512 stamps runs as two lanes (halves on
    two streams with their own lists, graphs and restrictions); every stamp
    gives the bits it gives in a smaller batch, which runs as one lane."""
    ctx, fit = _lane_fitter(gfo)
    two = []
    for pe in (4, 1):   # the count read every fourth iteration, and after every one
        print(f"600 stamps: two lanes, poll_every {pe}", flush=True)
        two.append(fit(list(range(600)), poll_every=pe))
        assert np.all(np.isfinite(two[-1][0])) and np.any(two[-1][1]["iters"] > 4)
    for lo_, hi_ in ((0, 300), (300, 600)):
        print(f"stamps {lo_}..{hi_ - 1}: one lane", flush=True)
        one = fit(list(range(lo_, hi_)))
        for t in two:
            _same_stamps(one, t, lo_, hi_)
    torch.cuda.synchronize()
    ctx.close()


@pytest.mark.parametrize("max_iter", [1, 3])
def test_two_lanes_iteration_cap(gfo, max_iter):
    """Two lanes stopped by a small iteration cap (before any stamp has
    converged, and between polls when the count is read every second
    iteration) give every stamp the bits of the same fit as one lane."""
    ctx, fit = _lane_fitter(gfo)
    for pe in (1, 2):
        print(f"600 stamps: two lanes, max_iter {max_iter}, poll_every {pe}", flush=True)
        two = fit(list(range(600)), max_iter=max_iter, poll_every=pe)
        assert np.all(two[1]["iters"] <= max_iter)
        for lo_, hi_ in ((0, 300), (300, 600)):
            print(f"stamps {lo_}..{hi_ - 1}: one lane", flush=True)
            _same_stamps(fit(list(range(lo_, hi_)), max_iter=max_iter, poll_every=pe), two, lo_, hi_)
    torch.cuda.synchronize()
    ctx.close()


def test_two_lanes_with_moves_repeatable():
    """An uneven batch (1024 stamps of 32..256 px, both FFT forms) in two
    lanes, with one-workgroup stamps moving to the multi-pass launches once
    few of their bucket remain (the default): one lane's chi^2 convolution
    runs while the other convolves its Jacobian images, so the two must not
    share scratch spectra.  Repeated fits of the same input give the same
    bits."""
    ctx = ops.Context(0)
    stamps = synth.c3(1024)
    n = len(stamps)
    batch = ops.Batch(ctx, [s.H for s in stamps], [s.W for s in stamps], [s.K for s in stamps], [1] * n)
    taps = to_dev(np.concatenate([s.psf.ravel() for s in stamps]), torch.float32)
    psf = ops.Psf(ctx, batch, taps, ops.GF_CONV_AUTO)
    forms = set(int(u) for u in psf.uses_fft)
    assert {1, 2} <= forms, forms
    truth = to_dev(np.concatenate([s.truth for s in stamps]), torch.float32)
    m = ops.model(ctx, batch, psf, truth, 5).cpu().numpy().astype(np.float64)
    off = batch.offsets["pix"]
    d, w = np.empty_like(m), np.empty_like(m)
    for i, s in enumerate(stamps):
        sl = slice(off[i], off[i] + s.H * s.W)
        dd, ww = synth.add_gaussian_noise(m[sl].reshape(s.H, s.W), s.noise_sigma, s.noise_seed)
        d[sl], w[sl] = dd.ravel(), ww.ravel()
    data, weight = to_dev(d, torch.float32), to_dev(w, torch.float32)
    lo = to_dev(np.concatenate([synth.bounds(1, s.H, s.W)[0] for s in stamps]), torch.float64)
    hi = to_dev(np.concatenate([synth.bounds(1, s.H, s.W)[1] for s in stamps]), torch.float64)
    start = to_dev(np.concatenate([s.start for s in stamps]), torch.float64)
    for pe in (4, 1):
        runs = []
        for r in range(3):
            print(f"1024 uneven stamps, poll_every {pe}: fit {r}", flush=True)
            th, info = ops.fit_lm(ctx, batch, psf, data, weight, start, lo=lo, hi=hi, ftol=1e-5, poll_every=pe)
            runs.append((th.cpu().numpy(), info))
        assert np.all(np.isfinite(runs[0][0])) and np.any(runs[0][1]["iters"] > 10)
        for th, info in runs[1:]:
            np.testing.assert_array_equal(th, runs[0][0])
            for f in ("chi2", "iters", "nfev", "njev", "status"):
                np.testing.assert_array_equal(info[f], runs[0][1][f], err_msg=f)
    torch.cuda.synchronize()
    ctx.close()
