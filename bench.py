"""Benchmark of the galaxy-fitting hot path on one MI355X.

Default workload (one 512x512 image, Sersic bulge + exponential disk, 65x65
Moffat PSF on a 576-point FFT grid, 15 free parameters, Poisson + read noise):
one step is one whole Levenberg-Marquardt fit from the seeded perturbed start
to the relative chi^2 tolerance 1e-5, run by gf_fit_lm on the device, i.e. one
pass of every stage of the hot path (parameter set-up, Sersic evaluation with
5x5 oversampling and its derivatives, FFT convolution, chi^2 and residual,
normal equations, FP64 solve and damping update).

  value   = model evaluations per second counted in output pixels (Mpix/s):
            512^2 x (trial evaluations + Jacobian evaluations) per fit / time
            per fit.  Every one of them runs steps 1-3 over the whole image.
  fits/s  = fits per second (reported beside it).

`--workload c4` runs the likelihood batch instead (1024 parameter vectors
against one 256x256 image with a 33x33 Moffat PSF; one step = steps 1-3 for all
vectors through gf_likelihood).

The roofline entry is for the kernel with the largest share of the step's GPU
time, measured with HIP events recorded by the library on the stream each
kernel is launched on (a separate, non-graph fit with per-kernel timing on).
The CPU baseline times the FP64 oracle on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (packed FMA)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5", "lines"], default="c2")
    ap.add_argument("--train-stamps", type=int, default=200_000, help="C5: rendered training stamps")
    ap.add_argument("--epochs", type=int, default=4, help="C5: training epochs")
    ap.add_argument("--mcmc-steps", type=int, default=2000, help="C4: Metropolis steps of the chain run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--breakdown", action="store_true", help="print the per-kernel breakdown to stderr")
    ap.add_argument("--calibrate-peaks", action="store_true",
                    help="only run the triad / FMA / transcendental probes and print the measured peaks")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB device buffer three times (reference for HBM byte counters)")
    return ap.parse_args()


# Algorithmic work per unit (see the roofline notes in the design document).
# Evaluation: FP32 operations per sub-sample and component, counting an FMA as
# two and a transcendental (log2 / exp2) as one.
EVAL_FLOP_PER_SUB = 17
EVAL_JAC_FLOP_PER_SUB = 35


def kernel_work(name, geo, launches_per_step):
    """(bound, algorithmic units per launch, unit) for a kernel of the step."""
    npix, npad, nch, ncomp, S, L, H = (geo[k] for k in ("npix", "npad", "nch", "ncomp", "S", "L", "H"))
    Lh = L // 2 + 1
    if name == "k_eval":
        return "alu", npad * ncomp * S * S * EVAL_FLOP_PER_SUB, "flop"
    if name == "k_eval_jac":
        return "alu", npad * ncomp * S * S * EVAL_JAC_FLOP_PER_SUB, "flop"
    if name == "k_chi2":
        # model read per pixel; data and weight per distinct image
        return "hbm", npix * 4 + geo.get("nimg", npix) * 8, "byte"
    if name == "k_gram":
        return "hbm", npix * (4 * nch + 8), "byte"
    if name == "k_line_lm":
        # FP32 operations of the whole fit (see line_fit_flops), one launch
        return "alu", geo["line_flops"], "flop"
    if name == "k_fft_irows_chi2":
        # inverse rows of the spectra in, data and weight per distinct image
        return "hbm", geo.get("chan_" + name, 1) * H * Lh * 8 + geo.get("nimg", npix) * 8, "byte"
    if name in ("k_fft_rows", "k_fft_cols", "k_fft_irows") and "fft_bytes" in geo:
        per_ch, once = geo["fft_bytes"][name]
        return "hbm", geo.get("chan_" + name, 1) * per_ch + once, "byte"
    if name in ("k_fft_rows", "k_fft_cols", "k_fft_irows"):
        c = geo.get("chan_" + name, 1)
        if name == "k_fft_rows":
            return "hbm", c * (npad * 4 + (npad // geo["Mw"]) * Lh * 8), "byte"
        if name == "k_fft_cols":
            return "hbm", c * ((npad // geo["Mw"]) * Lh * 8 + H * Lh * 8) + L * Lh * 8, "byte"
        return "hbm", c * (H * Lh * 8 + npix * 4), "byte"
    return None, 0, None


def run_c2(args, torch, ops, synth):
    dev = torch.device("cuda", 0)
    st = synth.c2()
    ctx = ops.Context(0)
    batch = ops.Batch(ctx, [st.H], [st.W], [st.K], [2])
    taps = torch.from_numpy(st.psf.astype(np.float32).ravel()).to(dev)
    psf = ops.Psf(ctx, batch, taps, ops.GF_CONV_FFT)
    # observation: the model at the truth (rendered by the library) plus noise
    truth32 = torch.from_numpy(st.truth.astype(np.float32)).to(dev)
    m_true = ops.model(ctx, batch, psf, truth32, 5).cpu().numpy().astype(np.float64).reshape(st.H, st.W)
    d, w = synth.add_poisson_read_noise(m_true, st.meta["read_noise"], st.meta["gain"], st.noise_seed)
    data = torch.from_numpy(d.astype(np.float32).ravel()).to(dev)
    weight = torch.from_numpy(w.astype(np.float32).ravel()).to(dev)
    lo, hi = synth.bounds(2, st.H, st.W)
    lo_t = torch.from_numpy(lo).to(dev)
    hi_t = torch.from_numpy(hi).to(dev)
    theta0 = torch.from_numpy(st.start).to(dev)
    opts = dict(ftol=1e-5, max_iter=100)

    def step(**kw):
        o = dict(opts)
        o.update(kw)
        return ops.fit_lm(ctx, batch, psf, data, weight, theta0, lo=lo_t, hi=hi_t, **o)

    # a fit takes well under a millisecond: 100 timed fits keep the host's
    # share of the timing noise small
    K = args.steps if args.steps is not None else 100
    W = args.warmup if args.warmup is not None else 5
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    # the result records stay on the device during the timed fits (as the
    # fitted parameters do) and are read after the timed region
    t0 = time.perf_counter()
    recs = []
    for _ in range(K):
        th, res = step(return_device=True)
        recs.append(res)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    infos = [ops.lm_info(r) for r in recs]
    info = infos[-1]
    nfev, njev, iters = int(info["nfev"][0]), int(info["njev"][0]), int(info["iters"][0])
    if any(int(i["nfev"][0]) != nfev or int(i["njev"][0]) != njev for i in infos):
        raise RuntimeError("fits of the same input took different paths")
    ms = t / K * 1e3
    npix = st.H * st.W
    mpix_s = (nfev + njev) * npix / (ms * 1e-3) / 1e6
    # per-kernel breakdown of one fit (no graph, events on the launching stream)
    from paper_1101_2254_amd import _lib
    _lib.gf_profile_start(ctx.ptr)
    step(use_graph=0)
    torch.cuda.synchronize()
    _lib.gf_profile_stop(ctx.ptr)
    prof = _lib.gf_profile_read(ctx.ptr)
    geo = dict(npix=npix, npad=(st.H + st.K - 1) * (st.W + st.K - 1), Mw=st.W + st.K - 1, H=st.H, nch=14, ncomp=2,
               S=5, L=psf.fft_side[0])
    result = dict(
        metric="model evals/sec (Mpix/s eval+PSF+χ²) and LM fits/sec at χ² rel tol 1e-5",
        value=round(mpix_s, 3), unit="Mpix/s", ms_per_step=round(ms, 4), fits_per_s=round(1e3 / ms, 3),
        lm=dict(iters=iters, nfev=nfev, njev=njev, status=int(info["status"][0]), chi2=float(info["chi2"][0]),
                chi2_per_dof=float(info["chi2"][0]) / (npix - 15)),
        config=dict(workload="C2: one 512x512 image, Sersic bulge + exponential disk, 65x65 Moffat PSF "
                             "(beta=3, FWHM=3 px), 576-point FFT convolution, 5x5 oversampling, 15-parameter "
                             "LM fit to chi2 rel tol 1e-5; one step = one whole fit",
                    image=[st.H, st.W], psf=st.K, fft_side=psf.fft_side[0], params=15, oversample=5),
    )
    result.update(steps=K, warmup=W)
    return result, prof, geo, dict(st=st, nfev=nfev, njev=njev, iters=iters, npix=npix)


def run_c3(args, torch, ops, synth):
    """4096 uneven single-Sersic stamps fitted in one gf_fit_lm call (ftol 1e-5)."""
    dev = torch.device("cuda", 0)
    stamps = synth.c3(4096)
    n = len(stamps)
    ctx = ops.Context(0)
    H = [s.H for s in stamps]
    K = [s.K for s in stamps]
    batch = ops.Batch(ctx, H, H, K, [1] * n)
    taps = torch.from_numpy(np.concatenate([s.psf.astype(np.float32).ravel() for s in stamps])).to(dev)
    psf = ops.Psf(ctx, batch, taps, ops.GF_CONV_AUTO)
    truth = torch.from_numpy(np.concatenate([s.truth for s in stamps]).astype(np.float32)).to(dev)
    m_true = ops.model(ctx, batch, psf, truth, 5).cpu().numpy().astype(np.float64)
    off = batch.offsets["pix"]
    d = np.empty_like(m_true)
    w = np.empty_like(m_true)
    for i, st in enumerate(stamps):
        sl = slice(off[i], off[i] + st.H * st.W)
        d[sl], w[sl] = synth.add_gaussian_noise(m_true[sl], st.noise_sigma, st.noise_seed)
    data = torch.from_numpy(d.astype(np.float32)).to(dev)
    weight = torch.from_numpy(w.astype(np.float32)).to(dev)
    lo = np.concatenate([synth.bounds(1, s.H, s.W)[0] for s in stamps])
    hi = np.concatenate([synth.bounds(1, s.H, s.W)[1] for s in stamps])
    lo_t, hi_t = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)
    theta0 = torch.from_numpy(np.concatenate([s.start for s in stamps])).to(dev)

    def step(**kw):
        o = dict(ftol=1e-5, max_iter=100)
        o.update(kw)
        return ops.fit_lm(ctx, batch, psf, data, weight, theta0, lo=lo_t, hi=hi_t, **o)

    K_ = args.steps if args.steps is not None else 5
    W = args.warmup if args.warmup is not None else 1
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K_):
        _, info = step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms = t / K_ * 1e3
    from paper_1101_2254_amd import _lib
    _lib.gf_profile_start(ctx.ptr)
    step(use_graph=0)
    torch.cuda.synchronize()
    _lib.gf_profile_stop(ctx.ptr)
    prof = _lib.gf_profile_read(ctx.ptr)
    npix = int(sum(s.H * s.W for s in stamps))
    npad = int(sum((s.H + s.K - 1) ** 2 for s in stamps))
    evals = int(info["nfev"].sum() + info["njev"].sum())
    result = dict(
        metric="model evals/sec (Mpix/s eval+PSF+χ²) and LM fits/sec at χ² rel tol 1e-5",
        value=round(n / (ms * 1e-3), 2), unit="fits/s", ms_per_step=round(ms, 3),
        mpix_per_s=round(evals / n * npix / n * n / (ms * 1e-3) / 1e6, 2),
        lm=dict(iters_mean=float(info["iters"].mean()), iters_max=int(info["iters"].max()),
                converged=float((info["status"] == 0).mean()), nfev=int(info["nfev"].sum()),
                njev=int(info["njev"].sum())),
        config=dict(workload="C3: 4096 uneven single-Sersic stamps (32..256 px, Gaussian/Moffat PSF 15..33 px), "
                             "one gf_fit_lm call to chi2 rel tol 1e-5; one step = the whole batch",
                    stamps=n, pixels=npix, oversample=5,
                    fft_stamps=int(sum(psf.uses_fft)), direct_stamps=int(n - sum(psf.uses_fft))),
    )
    fb = {"k_fft_rows": [0, 0], "k_fft_cols": [0, 0], "k_fft_irows": [0, 0]}
    for st, uf, L in zip(stamps, psf.uses_fft, psf.fft_side):
        if not uf:
            continue
        M, Lh = st.H + st.K - 1, L // 2 + 1
        fb["k_fft_rows"][0] += M * M * 4 + M * Lh * 8
        fb["k_fft_cols"][0] += M * Lh * 8 + st.H * Lh * 8
        fb["k_fft_cols"][1] += L * Lh * 8
        fb["k_fft_irows"][0] += st.H * Lh * 8 + st.H * st.W * 4
    geo = dict(npix=npix, npad=npad, Mw=1, H=1, nch=7, ncomp=1, S=5, L=2, fft_bytes=fb)
    result.update(steps=K_, warmup=W)
    return result, prof, geo, dict(stamps=stamps, info=info, npix=npix, nfev=int(info["nfev"].sum()),
                                   njev=int(info["njev"].sum()))


def run_c4(args, torch, ops, synth):
    dev = torch.device("cuda", 0)
    base = synth.c4_truth()
    nvec = 1024
    ctx = ops.Context(0)
    batch = ops.Batch(ctx, [256] * nvec, [256] * nvec, [33] * nvec, [1] * nvec, shared=True)
    taps = torch.from_numpy(base.psf.astype(np.float32).ravel()).to(dev)
    psf = ops.Psf(ctx, batch, taps, ops.GF_CONV_FFT)
    one = ops.Batch(ctx, [256], [256], [33], [1])
    psf1 = ops.Psf(ctx, one, taps, ops.GF_CONV_FFT)
    m_true = ops.model(ctx, one, psf1, torch.from_numpy(base.truth.astype(np.float32)).to(dev), 5)
    d, w = synth.add_gaussian_noise(m_true.cpu().numpy().astype(np.float64).reshape(256, 256), base.noise_sigma,
                                    base.noise_seed)
    data = torch.from_numpy(d.astype(np.float32).ravel()).to(dev)
    weight = torch.from_numpy(w.astype(np.float32).ravel()).to(dev)
    K = args.steps if args.steps is not None else 50
    W = args.warmup if args.warmup is not None else 3
    thetas = [torch.from_numpy(synth.c4_vectors(s, nvec).astype(np.float32).ravel()).to(dev) for s in range(K + W)]
    work = ops.likelihood_workspace(ctx, batch, psf)
    out = torch.empty((nvec, 2), dtype=torch.float32, device=dev)
    for s in range(W):
        ops.likelihood(ctx, batch, psf, thetas[s], data, weight, 5, work=work, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        ops.likelihood(ctx, batch, psf, thetas[W + s], data, weight, 5, work=work, out=out)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms = t / K * 1e3
    npix = 256 * 256 * nvec
    # Metropolis chains on the same batch: one chain per vector, started from
    # this step's vectors, 2000 steps (each step = steps 1-3 for all chains)
    n_mc = args.mcmc_steps
    scale = torch.from_numpy(np.tile(np.abs(base.truth) * 1e-4 + 1e-6, nvec)).to(dev)
    lo_b, hi_b = synth.bounds(1, 256, 256)
    lo_m = torch.from_numpy(np.tile(lo_b, nvec)).to(dev)
    hi_m = torch.from_numpy(np.tile(hi_b, nvec)).to(dev)
    th_mc = thetas[0].double()
    ops.mcmc_run(ctx, batch, psf, data, weight, th_mc, scale, 10, key=(4004, 1), lo=lo_m, hi=hi_m,
                 keep_samples=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, c2_mc, _, acc_mc = ops.mcmc_run(ctx, batch, psf, data, weight, th_mc, scale, n_mc, key=(4004, 1), stream=1,
                                       lo=lo_m, hi=hi_m, keep_samples=False)
    torch.cuda.synchronize()
    t_mc = time.perf_counter() - t0
    mcmc = dict(chains=nvec, steps=n_mc, ms_per_step=round(t_mc / n_mc * 1e3, 4),
                mpix_per_s=round(npix * n_mc / t_mc / 1e6, 1),
                accept_rate=round(float(acc_mc.double().mean().item()) / n_mc, 4),
                proposal="theta' = theta + (1e-4 |theta_true| + 1e-6) z, flat prior on the fit bounds")
    from paper_1101_2254_amd import _lib
    _lib.gf_profile_start(ctx.ptr)
    ops.likelihood(ctx, batch, psf, thetas[0], data, weight, 5, work=work, out=out)
    torch.cuda.synchronize()
    _lib.gf_profile_stop(ctx.ptr)
    prof = _lib.gf_profile_read(ctx.ptr)
    # steps 2 and 3 also as the separate entry points (gf_convolve_psf, then
    # gf_chi2 on its output), each timed by the library's per-kernel events
    mp = ops.eval_model(ctx, batch, thetas[0], 5)
    mc = ops.convolve_psf(ctx, batch, psf, mp)
    ops.chi2(ctx, batch, mc, thetas[0], data, weight)
    torch.cuda.synchronize()
    _lib.gf_profile_start(ctx.ptr)
    for _ in range(5):
        ops.convolve_psf(ctx, batch, psf, mp, out=mc)
        ops.chi2(ctx, batch, mc, thetas[0], data, weight)
    torch.cuda.synchronize()
    _lib.gf_profile_stop(ctx.ptr)
    sep_prof = _lib.gf_profile_read(ctx.ptr)
    del mp, mc
    geo = dict(npix=npix, npad=288 * 288 * nvec, Mw=288, H=256 * nvec, nch=1, ncomp=1, S=5, L=psf.fft_side[0],
               nimg=256 * 256, separate=sep_prof)
    result = dict(
        metric="model evals/sec (Mpix/s eval+PSF+χ²) and LM fits/sec at χ² rel tol 1e-5",
        value=round(npix / (ms * 1e-3) / 1e6, 3), unit="Mpix/s", ms_per_step=round(ms, 4),
        config=dict(workload="C4: likelihood batch, 1024 parameter vectors x one 256x256 image, 33x33 Moffat PSF, "
                             "288-point FFT, 5x5 oversampling; one step = steps 1-3 for all vectors",
                    image=[256, 256], psf=33, fft_side=psf.fft_side[0], vectors=nvec, oversample=5),
        mcmc=mcmc,
    )
    result.update(steps=K, warmup=W)
    return result, prof, geo, dict(base=base, thetas_host=synth.c4_vectors(W, nvec), npix=npix)


# Proposal network work per stamp (multiply-adds of the four 3x3 stride-2
# convolutions at 128 x 128 input plus the two dense layers), times two for
# FLOPs; a training step costs about three forward passes.
CNN_MAC_PER_STAMP = (64 * 64 * 32 * 9 * 1 + 32 * 32 * 32 * 9 * 32 + 16 * 16 * 64 * 9 * 32 + 8 * 8 * 64 * 9 * 64
                     + 4096 * 256 + 256 * 8)
BF16_PEAK_TFLOPS = 2500.0


def run_c5(args, torch, ops, synth):
    """Learned proposal: train on stamps rendered on the device, then fit 4096
    fresh 128x128 stamps by LM from the network's proposals and from the
    image-moment default guess.  One step = proposal + LM for the batch."""
    from paper_1101_2254_amd import proposal as PR
    from paper_1101_2254_amd import _lib
    dev = torch.device("cuda", 0)
    ctx = ops.Context(0)
    side, nev = 128, 4096
    t0 = time.perf_counter()
    train = PR.RenderedSet(ctx, synth.psf_bank(2048, 2000), args.train_stamps, side, seed=2000)
    torch.cuda.synchronize()
    t_render = time.perf_counter() - t0
    net = PR.ProposalNet(ctx, side, max_batch=256)
    net.init(2000)
    print(f"bench: rendered {args.train_stamps} stamps in {t_render:.2f} s; training {args.epochs} epochs",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    losses = PR.train(net, train, epochs=args.epochs, batch=256, lr=2e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps_trained = net.steps
    del train
    ev = PR.RenderedSet(ctx, synth.psf_bank(nev, 3000), nev, side, seed=3000)
    data = ev.noisy(0, nev, epoch=0).clone()
    weight = torch.full_like(data, 1.0 / 0.02 ** 2)
    lo, hi = synth.bounds(1, side, side)
    lo_t = torch.from_numpy(np.tile(lo, nev)).to(dev)
    hi_t = torch.from_numpy(np.tile(hi, nev)).to(dev)

    def fit(start, **kw):
        return ops.fit_lm(ctx, ev.batch, ev.psf, data, weight, start, lo=lo_t, hi=hi_t, ftol=1e-5, max_iter=100,
                          **kw)

    def step_cnn(**kw):
        return fit(net.predict(data).reshape(-1).contiguous(), **kw)

    def step_default():
        return fit(PR.moments_guess(ctx, ev.batch, data))

    K_ = args.steps if args.steps is not None else 5
    W = args.warmup if args.warmup is not None else 1
    times = {}
    infos = {}
    for name, fn in (("default", step_default), ("cnn", step_cnn)):
        for _ in range(W):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K_):
            _, infos[name] = fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / K_
    # training GEMM rate from the library's per-kernel timing of one step
    xb = ev.noisy(0, 256, epoch=7)
    tb = PR.encode(ctx, ev.theta[:256].reshape(-1), side)
    net.train_step(xb, tb, 1e-6)
    torch.cuda.synchronize()
    _lib.gf_profile_start(ctx.ptr)
    net.train_step(xb, tb, 1e-6)
    torch.cuda.synchronize()
    _lib.gf_profile_stop(ctx.ptr)
    tprof = _lib.gf_profile_read(ctx.ptr)
    _lib.gf_profile_start(ctx.ptr)
    step_cnn(use_graph=0)
    torch.cuda.synchronize()
    _lib.gf_profile_stop(ctx.ptr)
    prof = _lib.gf_profile_read(ctx.ptr)
    ic, idf = infos["cnn"], infos["default"]
    rel = (ic["chi2"] - idf["chi2"]) / idf["chi2"]
    gemm_ms = tprof.get("k_gemm_bf16", (0, 0.0))[1]
    step_ms = sum(v[1] for v in tprof.values())
    train_flop = 3 * 2 * CNN_MAC_PER_STAMP * 256
    result = dict(
        metric="model evals/sec (Mpix/s eval+PSF+χ²) and LM fits/sec at χ² rel tol 1e-5",
        value=round(nev / times["cnn"], 2), unit="fits/s", ms_per_step=round(times["cnn"] * 1e3, 3),
        fits_per_s=round(nev / times["cnn"], 2),
        lm=dict(iters_mean=float(ic["iters"].mean()), converged=float((ic["status"] == 0).mean())),
        c5=dict(
            default_fits_per_s=round(nev / times["default"], 2),
            speedup_vs_default=round(times["default"] / times["cnn"], 3),
            iters_mean_cnn=float(ic["iters"].mean()), iters_mean_default=float(idf["iters"].mean()),
            converged_cnn=float((ic["status"] == 0).mean()), converged_default=float((idf["status"] == 0).mean()),
            equal_chi2_frac=float(np.mean(np.abs(rel) <= 1e-5)), cnn_lower_chi2_frac=float(np.mean(rel < -1e-5)),
            default_lower_chi2_frac=float(np.mean(rel > 1e-5)),
            train=dict(stamps=args.train_stamps, epochs=args.epochs, steps=steps_trained, batch=256,
                       render_s=round(t_render, 3), train_s=round(t_train, 3),
                       stamps_per_s=round(args.epochs * args.train_stamps / t_train, 1),
                       loss_per_epoch=[round(v, 5) for v in losses],
                       step_kernel_ms=round(step_ms, 4), gemm_ms=round(gemm_ms, 4),
                       gemm_tflops=round(train_flop / (gemm_ms * 1e-3) / 1e12, 2) if gemm_ms else None,
                       gemm_frac_bf16_peak=round(train_flop / (gemm_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4)
                       if gemm_ms else None)),
        config=dict(workload="C5: 4096 fresh 128x128 single-Sersic stamps (uneven-batch priors, Gaussian/Moffat "
                             "PSF 15..33 px, noise 0.02); one step = network proposal + one gf_fit_lm call to chi2 "
                             "rel tol 1e-5", stamps=nev, side=side, oversample=5),
    )
    npix = nev * side * side
    fb = {"k_fft_rows": [0, 0], "k_fft_cols": [0, 0], "k_fft_irows": [0, 0]}
    geo = dict(npix=npix, npad=npix, Mw=1, H=1, nch=7, ncomp=1, S=5, L=2, fft_bytes=fb)
    result.update(steps=K_, warmup=W)
    return result, prof, geo, dict(info=ic, nfev=int(ic["nfev"].sum()), njev=int(ic["njev"].sum()))


# Algorithmic FP32 operations of one line fit, counting an FMA as two and an
# exp2 as one: per padded channel, sub-sample and line 6 for the model
# (offset, square, scale, exp2, accumulate) and 10 with the three
# derivatives; per output channel 2 K per convolved plane; the Gram matrix
# 2 (P + 1)(P + 2)/2 per output channel.
def line_fit_flops(N, K, nl, S, nfev, njev):
    P = 3 * nl + 1
    npad = N + K - 1
    model = npad * S * nl * 6 + N * 2 * K + 4 * N
    jac = npad * S * nl * 10 + N * 2 * K * P + N * (P + 1) * (P + 2)
    return nfev * model + njev * jac


def run_lines(args, torch, ops, synth):
    dev = torch.device("cuda", 0)
    n = 65536
    spectra = synth.line_batch(n)
    ctx = ops.Context(0)
    lb = ops.LineBatch(ctx, [s.N for s in spectra], [s.K for s in spectra], [s.nlines for s in spectra])
    lsf = torch.from_numpy(np.concatenate([s.lsf for s in spectra]).astype(np.float32)).to(dev)
    truth = torch.from_numpy(np.concatenate([s.truth for s in spectra]).astype(np.float32)).to(dev)
    start = torch.from_numpy(np.concatenate([s.start for s in spectra])).to(dev)
    lo = torch.from_numpy(np.concatenate([synth.line_bounds(s.nlines, s.N)[0] for s in spectra])).to(dev)
    hi = torch.from_numpy(np.concatenate([synth.line_bounds(s.nlines, s.N)[1] for s in spectra])).to(dev)
    # observation: the library's model at the truth plus seeded noise
    m_true = ops.line_model(ctx, lb, lsf, truth, 5).cpu().numpy().astype(np.float64)
    d, w = synth.add_noise_1d(m_true, 0.05, synth.SEED_BASE + 60)
    data = torch.from_numpy(d.astype(np.float32)).to(dev)
    weight = torch.from_numpy(w.astype(np.float32)).to(dev)

    def step():
        return ops.line_fit_lm(ctx, lb, lsf, data, weight, start, lo=lo, hi=hi, ftol=1e-5, max_iter=100,
                               return_device=True)

    K = args.steps if args.steps is not None else 20
    W = args.warmup if args.warmup is not None else 3
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        th, res = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / K * 1e3
    info = ops.lm_info(res)
    from paper_1101_2254_amd import _lib
    _lib.gf_profile_start(ctx.ptr)
    step()
    torch.cuda.synchronize()
    _lib.gf_profile_stop(ctx.ptr)
    prof = _lib.gf_profile_read(ctx.ptr)
    S = 5
    flops = sum(line_fit_flops(s.N, s.K, s.nlines, S, int(info["nfev"][i]), int(info["njev"][i]))
                for i, s in enumerate(spectra))
    chan_evals = sum(s.N * (int(info["nfev"][i]) + int(info["njev"][i])) for i, s in enumerate(spectra))
    nch = sum(s.N for s in spectra)
    result = dict(
        metric="model evals/sec (Mpix/s eval+PSF+χ²) and LM fits/sec at χ² rel tol 1e-5",
        value=round(n / (ms * 1e-3), 2), unit="fits/s", ms_per_step=round(ms, 4),
        mpix_per_s=round(chan_evals / (ms * 1e-3) / 1e6, 2),
        lm=dict(iters_mean=float(info["iters"].mean()), iters_max=int(info["iters"].max()),
                converged=float((info["status"] == 0).mean()), nfev=int(info["nfev"].sum()),
                njev=int(info["njev"].sum())),
        config=dict(workload="lines: 65536 spectra of 256..2048 channels with 1..3 Gaussian emission lines and a "
                             "continuum, 7..21-tap Gaussian LSF, 5x sub-sampling, one gf_line_fit_lm call to chi2 "
                             "rel tol 1e-5; one step = the whole batch",
                    spectra=n, channels=nch, oversample=S))
    geo = dict(npix=nch, npad=nch, Mw=1, H=1, nch=1, ncomp=1, S=S, L=2, line_flops=flops)
    result.update(steps=K, warmup=W)
    return result, prof, geo, dict(spectra=spectra, info=info, data=d, weight=w)


def cpu_baseline_lines(extra, seconds):
    """The line oracle fitting the same spectra (the same observations, as
    FP32 values) one after another within the time budget."""
    from oracle import line_ref as LR
    import synth
    spectra, d, w = extra["spectra"], extra["data"].astype(np.float32), extra["weight"].astype(np.float32)
    offs = np.cumsum([0] + [s.N for s in spectra])
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds and n < len(spectra):
        s = spectra[n]
        lo, hi = synth.line_bounds(s.nlines, s.N)
        LR.fit_lm(s.start, s.lsf.astype(np.float32).astype(np.float64), d[offs[n]:offs[n + 1]].astype(np.float64),
                  w[offs[n]:offs[n + 1]].astype(np.float64), 5, lo=lo, hi=hi, ftol=1e-5, max_iter=100)
        n += 1
    t = time.perf_counter() - t0
    return dict(value=round(n / t, 3), unit="fits/s", cores=1, kind="oracle",
                sample=f"numpy FP64 line oracle fitting the first {n} spectra of the batch to ftol 1e-5, "
                       f"{t:.1f} s on one thread")


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by the copy calibration: fetch x2, write x1), as
# summarised in profiles/*_hbm_traffic.md: bytes = once + per_channel x
# channels per launch.  Valid only while the kernel source is the one the
# counters were taken on (first 16 hex digits of its SHA-256).
TRAFFIC = {
    "c2": {
        "k_eval_jac": dict(source="paper_1101_2254_amd/csrc/k_eval.hip", sha16="524bd17134a451f8", once=1.8800e+07,
                           per_channel=0.0),
        "k_fft_cols": dict(source="paper_1101_2254_amd/csrc/k_fft.hip", sha16="e5ad3e6d0c9bfbf0", once=1.5038e+06,
                           per_channel=2.8225e+06),
        "summary": "profiles/c2_fit_hbm_traffic.md"},
    "c4": {
        "k_eval": dict(source="paper_1101_2254_amd/csrc/k_eval.hip", sha16="524bd17134a451f8", once=3.8624e+08,
                       per_channel=0.0),
        "summary": "profiles/c4_likelihood_hbm_traffic.md"},
}


def stage_roofline(prof, geo):
    """Steps 2 and 3 of the likelihood batch as one fused stage (the chi^2
    is reduced in the inverse-row FFT pass, so the convolved model never
    reaches HBM), with the algorithmic bytes of its definition: read the
    padded model, data and weight once per distinct image, the OTF once.
    The FFT's own spectra traffic is not counted here (it is in the
    per-kernel figures of `stages`)."""
    out = {}
    L = geo.get("L", 0)
    ks = ("k_fft_rows", "k_fft_cols", "k_fft_irows_chi2")
    if L > 2 and all(k in prof for k in ks):
        n = prof["k_fft_rows"][0]
        t = sum(prof[k][1] / prof[k][0] for k in ks) * 1e-3
        b = 4 * geo["npad"] + 8 * geo.get("nimg", geo["npix"]) + L * (L // 2 + 1) * 8
        out["convolution_chi2"] = dict(kernels=list(ks), launches=n, bytes_per_launch=int(b),
                                       us_per_launch=round(t * 1e6, 2), gbs=round(b / t / 1e9, 1),
                                       frac=round(b / t / 1e9 / HBM_PEAK_GBS, 4))
    sep = geo.get("separate")
    if sep:
        # the separate entry points: convolution = padded model read + stamp
        # written + OTF once; chi^2 = model read + data and weight once
        ks = ("k_fft_rows", "k_fft_cols", "k_fft_irows")
        if all(k in sep for k in ks):
            n = sep["k_fft_rows"][0]
            t = sum(sep[k][1] / sep[k][0] for k in ks) * 1e-3
            b = 4 * geo["npad"] + 4 * geo["npix"] + L * (L // 2 + 1) * 8
            out["convolution"] = dict(kernels=list(ks), launches=n, bytes_per_launch=int(b),
                                      us_per_launch=round(t * 1e6, 2), gbs=round(b / t / 1e9, 1),
                                      frac=round(b / t / 1e9 / HBM_PEAK_GBS, 4))
        # (large batches reduce each stamp in one launch: no k_pair_final)
        ks = tuple(k for k in ("k_chi2", "k_pair_final") if k in sep)
        if "k_chi2" in sep:
            n = sep["k_chi2"][0]
            t = sum(sep[k][1] / sep[k][0] for k in ks) * 1e-3
            b = 4 * geo["npix"] + 8 * geo.get("nimg", geo["npix"])
            out["chi2"] = dict(kernels=list(ks), launches=n, bytes_per_launch=int(b), us_per_launch=round(t * 1e6, 2),
                               gbs=round(b / t / 1e9, 1), frac=round(b / t / 1e9 / HBM_PEAK_GBS, 4))
    return out


def measured_traffic(workload, rl, geo):
    import hashlib
    t = TRAFFIC.get(workload, {}).get(rl.get("kernel"))
    if not t:
        return None
    try:
        with open(os.path.join(ROOT, t["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha16"]:
                return None
    except OSError:
        return None
    return round(t["once"] + t["per_channel"] * geo.get("chan_" + rl["kernel"], 1), 0)


def roofline(prof, geo):
    total = sum(v[1] for v in prof.values())
    name = max(prof, key=lambda k: prof[k][1])
    launches, tot_ms = prof[name]
    bound, units, what = kernel_work(name, geo, launches)
    avg_s = tot_ms / launches * 1e-3
    stages = {}
    for k, (n, t) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        b, u, wu = kernel_work(k, geo, n)
        e = dict(launches=n, ms_total=round(t, 4), share=round(t / total, 4))
        if b == "hbm":
            e.update(bound="hbm", gbs=round(u / (t / n * 1e-3) / 1e9, 1), frac=round(u / (t / n * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
        elif b == "alu":
            e.update(bound="alu", tflops=round(u / (t / n * 1e-3) / 1e12, 2),
                     frac=round(u / (t / n * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4))
        stages[k] = e
    if bound == "hbm":
        ach = units / avg_s / 1e9
        rl = dict(bound="hbm", kernel=name, achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                  frac=round(ach / HBM_PEAK_GBS, 4), traffic=None)
    else:
        ach = units / avg_s / 1e12
        rl = dict(bound="alu", kernel=name, achieved=round(ach, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                  frac=round(ach / FP32_PEAK_TFLOPS, 4), traffic=None)
    rl["avg_launch_us"] = round(avg_s * 1e6, 2)
    return rl, stages


def cpu_baseline_c2(extra, seconds):
    """The oracle on its own rendering of the same observation (FP64 model at
    the FP32 truth, the same seeded noise): the first LM iterations of the fit."""
    from oracle import gfo
    import synth
    st = extra["st"]
    threads = os.cpu_count() or 1
    gfo.set_threads(threads)
    lo, hi = synth.bounds(2, st.H, st.W)
    psf = st.psf.astype(np.float32).astype(np.float64)
    m_true = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64), psf, 5)
    d, w = synth.add_poisson_read_noise(m_true, st.meta["read_noise"], st.meta["gain"], st.noise_seed)
    d = d.astype(np.float32).astype(np.float64)
    w = w.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    iters = evals = 0
    n_it = 1
    while True:
        _, info = gfo.fit_lm(st.start, psf, d, w, 5, lo=lo, hi=hi, ftol=1e-5, max_iter=n_it)
        evals += info["nfev"] + info["njev"]
        iters += info["iters"]
        if time.perf_counter() - t0 >= seconds or n_it >= 8:
            break
        n_it += 1
    t = time.perf_counter() - t0
    mpix = evals * extra["npix"] / t / 1e6
    return dict(value=round(mpix, 5), unit="Mpix/s", cores=gfo.get_threads(), kind="oracle",
                sample=f"FP64 oracle LM on its own rendering of the same 512x512 observation: {iters} iterations "
                       f"in runs of 1..{n_it} iterations ({evals} model + Jacobian evaluations, direct "
                       f"convolution), {t:.1f} s on {gfo.get_threads()} threads",
                fits_per_s_est=round(1.0 / (t / evals * (extra["nfev"] + extra["njev"])), 6))


def cpu_baseline_c4(extra, seconds):
    """The oracle on its own rendering of the same image: steps 1-3 for as many
    of the step's parameter vectors as fit in the time budget."""
    from oracle import gfo
    import synth
    threads = os.cpu_count() or 1
    gfo.set_threads(threads)
    base = extra["base"]
    psf = base.psf.astype(np.float32).astype(np.float64)
    m_true = gfo.model(256, 256, base.truth.astype(np.float32).astype(np.float64), psf, 5)
    d, w = synth.add_gaussian_noise(m_true, base.noise_sigma, base.noise_seed)
    d = d.astype(np.float32).astype(np.float64)
    w = w.astype(np.float32).astype(np.float64)
    th = extra["thetas_host"].astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds and n < th.shape[0]:
        gfo.chi2(d, w, gfo.model(256, 256, th[n], psf, 5))
        n += 1
    t = time.perf_counter() - t0
    return dict(value=round(n * 256 * 256 / t / 1e6, 5), unit="Mpix/s", cores=gfo.get_threads(), kind="oracle",
                sample=f"FP64 oracle eval + direct convolution + chi2 of {n} of the step's parameter vectors on "
                       f"its own rendering of the image, {t:.1f} s on {gfo.get_threads()} threads")


def cpu_baseline_c3(extra, seconds):
    """Stratified sample: per stamp size, the oracle's first LM iteration on its
    own rendering of one stamp of that size, scaled by the GPU run's mean
    iteration count for that size (extrapolated)."""
    from oracle import gfo
    import synth
    gfo.set_threads(os.cpu_count() or 1)
    stamps, info = extra["stamps"], extra["info"]
    total = 0.0
    used = []
    t_all = time.perf_counter()
    for N in synth.C3_SIZES:
        idx = [i for i, st in enumerate(stamps) if st.H == N]
        if not idx:
            continue
        st = stamps[idx[0]]
        psf = st.psf.astype(np.float32).astype(np.float64)
        m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64), psf, 5)
        d, w = synth.add_gaussian_noise(m, st.noise_sigma, st.noise_seed)
        lo, hi = synth.bounds(1, st.H, st.W)
        t0 = time.perf_counter()
        gfo.fit_lm(st.start, psf, d.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64),
                   5, lo=lo, hi=hi, ftol=1e-5, max_iter=1)
        t1 = time.perf_counter() - t0
        iters = float(np.mean(info["iters"][idx]))
        total += t1 * iters * len(idx)
        used.append(f"{N}:{t1 * 1e3:.0f}ms")
        if time.perf_counter() - t_all > seconds * 4:
            break
    return dict(value=round(len(stamps) / total, 4), unit="fits/s", cores=gfo.get_threads(), kind="oracle",
                sample="extrapolated: one oracle LM iteration (start evaluation + Jacobian + step) per stamp size "
                       "on its own rendering, times the GPU run's mean iterations per size and the stamps per size ("
                       + ", ".join(used) + ")")


def cpu_baseline_c5(extra, seconds):
    """One oracle LM iteration on its own rendering of a 128x128 C5-like
    stamp (one per PSF size class), times the GPU run's mean iterations of
    the network-seeded fits (extrapolated to the 4096-stamp batch)."""
    from oracle import gfo
    import synth
    gfo.set_threads(os.cpu_count() or 1)
    info = extra["info"]
    g = synth.rng(3000)
    ts = []
    t_all = time.perf_counter()
    for i in range(4):
        st = synth.c3_stamp(g, 128, i, 3000)
        psf = st.psf.astype(np.float32).astype(np.float64)
        m = gfo.model(128, 128, st.truth, psf, 5)
        d, w = synth.add_gaussian_noise(m, 0.02, 3000 + i)
        lo, hi = synth.bounds(1, 128, 128)
        t0 = time.perf_counter()
        gfo.fit_lm(st.start, psf, d, w, 5, lo=lo, hi=hi, ftol=1e-5, max_iter=1)
        ts.append(time.perf_counter() - t0)
        if time.perf_counter() - t_all > seconds:
            break
    per_iter = float(np.mean(ts))
    total = per_iter * float(info["iters"].mean()) * len(info)
    return dict(value=round(len(info) / total, 4), unit="fits/s", cores=gfo.get_threads(), kind="oracle",
                sample=f"extrapolated: {len(ts)} oracle LM iterations on 128x128 stamps "
                       f"(mean {per_iter * 1e3:.0f} ms) x mean GPU iterations x 4096 stamps")


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py: the library runs on one GPU; --gpus {max(args.gpus, world)} is not supported "
              "(the hot path shards as described in the design notes, but only the one-GPU kernel is built)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1101_2254_amd import ops
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=src.numel() * 4, copies=3)))
        return
    if args.calibrate_peaks:
        from paper_1101_2254_amd import _lib
        ctx = ops.Context(0)
        ctx.bind_stream()
        out = dict(triad_gbs=_lib.gf_probe(ctx.ptr, 0, 1 << 28, 10), fma_tflops=_lib.gf_probe(ctx.ptr, 1, 4096, 5),
                   transcendental_gops=_lib.gf_probe(ctx.ptr, 2, 2048, 5))
        out["triad_frac_of_8tbs"] = round(out["triad_gbs"] / HBM_PEAK_GBS, 4)
        print(json.dumps(out))
        return
    print(f"bench: workload {args.workload}", file=sys.stderr, flush=True)
    if args.workload == "c2":
        result, prof, geo, extra = run_c2(args, torch, ops, synth)
    elif args.workload == "c3":
        result, prof, geo, extra = run_c3(args, torch, ops, synth)
    elif args.workload == "c5":
        result, prof, geo, extra = run_c5(args, torch, ops, synth)
    elif args.workload == "lines":
        result, prof, geo, extra = run_lines(args, torch, ops, synth)
    else:
        result, prof, geo, extra = run_c4(args, torch, ops, synth)
    geo["chan_k_fft_rows"] = geo["chan_k_fft_cols"] = geo["chan_k_fft_irows"] = geo["chan_k_fft_irows_chi2"] = 1
    if args.workload in ("c2", "c3", "c5"):
        # per fit the row and column passes run 7 n_comp channels (Jacobian)
        # and 1 channel (trial) per launch: use the average over the launches
        # of the profiled fit; the plain inverse-row pass runs only for the
        # Jacobian, the fused one only for the trial points (a speculative
        # fit has no one-channel launches)
        n_jac = prof.get("k_eval_jac", (0, 0.0))[0]
        n_trial = prof.get("k_fft_irows_chi2", (0, 0.0))[0]
        nch = 14 if args.workload == "c2" else 7
        avg = (nch * n_jac + 1 * n_trial) / max(n_jac + n_trial, 1)
        for k in ("rows", "cols"):
            geo["chan_k_fft_" + k] = avg
        geo["chan_k_fft_irows"] = nch
    rl, stages = roofline(prof, geo)
    rl["traffic"] = measured_traffic(args.workload, rl, geo)
    stage_rl = stage_roofline(prof, geo) if args.workload == "c4" else {}
    if rl["traffic"] is not None:
        rl["traffic_source"] = TRAFFIC[args.workload]["summary"]
    if args.workload in ("c3", "c5"):
        # finished stamps skip their work units, so per-launch bytes of the
        # whole batch overstate what a launch moves: report times only
        for k in stages:
            for f in ("bound", "gbs", "tflops", "frac"):
                stages[k].pop(f, None)
        rl = dict(bound=None, kernel=rl["kernel"], achieved=None, peak=None, unit=None, frac=None, traffic=None,
                  avg_launch_us=rl["avg_launch_us"],
                  note="per-launch work varies as stamps finish; see the C2 and C4 workloads for rooflines")
    print(f"bench: {result['value']} {result['unit']}, {result['ms_per_step']} ms/step", file=sys.stderr,
          flush=True)
    if args.breakdown:
        print(json.dumps(stages, indent=1), file=sys.stderr)
    out = dict(metric=result["metric"], value=result["value"], unit=result["unit"], n_gpus=1,
               steps=result.pop("steps"), warmup=result.pop("warmup"), ms_per_step=result["ms_per_step"],
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data=("synthetic (seeded; stamps rendered by the library from on-device Philox4x64-10 prior draws and "
                     "noise)" if args.workload == "c5" else
                     "synthetic (seeded; spectra rendered by the library, noise from numpy PCG64)"
                     if args.workload == "lines" else
                     "synthetic (seeded; Sersic stamps rendered by the library, noise from numpy PCG64)"),
               config=result["config"], roofline=rl)
    for k in ("fits_per_s", "lm", "mpix_per_s", "c5", "mcmc"):
        if k in result:
            out[k] = result[k]
    out["stages"] = stages
    if stage_rl:
        out["stage_roofline"] = stage_rl
    if not args.no_cpu:
        if args.workload == "c2":
            out["cpu_baseline"] = cpu_baseline_c2(extra, args.cpu_seconds)
        elif args.workload == "c3":
            out["cpu_baseline"] = cpu_baseline_c3(extra, args.cpu_seconds)
        elif args.workload == "c5":
            out["cpu_baseline"] = cpu_baseline_c5(extra, args.cpu_seconds)
        elif args.workload == "lines":
            out["cpu_baseline"] = cpu_baseline_lines(extra, args.cpu_seconds)
        else:
            out["cpu_baseline"] = cpu_baseline_c4(extra, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
