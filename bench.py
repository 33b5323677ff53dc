"""Benchmark of the galaxy-fitting hot path on one MI355X.

Default run (no --workload): the uneven batch is the headline and the other
single-GPU workloads are nested in the same JSON line, each with its own
timing and roofline entry.

  headline  C3: 4096 single-Sersic stamps of 32..256 px (Gaussian/Moffat PSFs
            of 15..33 px) fitted by one gf_fit_lm call to the relative chi^2
            tolerance 1e-5.  One step = the whole batch (every stage of the
            hot path: parameter set-up, Sersic evaluation with 5x5
            oversampling and its derivatives, FFT convolution, chi^2, normal
            equations, FP64 solve and damping update).
            value = fits/s; mpix_per_s counts the steps 1-3 passes that ran
            (start point, trial points and Jacobians) in stamp pixels.
  c4        likelihood batch: 1024 parameter vectors x one 256 x 256 image with
            a 33 x 33 Moffat PSF; one step = steps 1-3 for all vectors;
            value = Mpix/s.
  c2        one 512 x 512 bulge + disk image, 65 x 65 Moffat PSF, 15
            parameters; one step = one whole fit; value = fits/s, mpix_per_s
            counts the evaluation passes the fit ran.
  c1        one 64 x 64 stamp, 8 parameters; latency: ms per whole fit.
  cube      256 integral-field cubes (32..64 spaxels square, 64 channels) of
            rotating disk galaxies, 12-parameter fits by one gf_cube_fit_lm
            call; value = fits/s, mvox_per_s counts the evaluation passes.

`--workload c3|c4|c2|c1|c5|lines|cube` runs one workload alone (its line has the
same layout as the headline).  `--steps` and `--warmup` apply to the headline
(or to the one workload); the nested workloads use their own defaults.

Rooflines: the dominant kernel of each workload's profiled step (per-kernel
HIP events recorded by the library on the stream each kernel is launched
on), its algorithmic bytes or operations per launch divided by its average
launch time, against the MI355X spec peaks (HBM 8 TB/s, FP32 157.3 TFLOP/s);
the measured triad, unpacked-FMA and transcendental rates are reported
beside.  For the uneven batch the profile is its first LM iteration, where
every stamp is active and the work per launch is known.  `stage_roofline`
gives steps 2 and 3 with their definitional bytes (convolution: padded model
read, stamp written, OTF once; with chi^2: padded model, data and weight
read, OTF once).

CPU baseline: the FP64 oracle (rebuilt -O3 -march=native for the host) on a
bounded sample of each workload, on one thread and on all host cores.
"""
from __future__ import annotations

import argparse
import hashlib
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
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 matrix
# the library's tuning file (FFT form per side, measured on first use)
TUNE_FILE = os.path.join(ROOT, "bench_out", "gf_tune.json")
METRIC = "model evals/sec (Mpix/s eval+PSF+χ²) and LM fits/sec at χ² rel tol 1e-5"

# Algorithmic FP32 operations per sub-sample and component (an FMA counts
# two, a log2 or exp2 one): the model 17, the model with its seven
# derivatives 35.
EVAL_FLOP_PER_SUB = 17
EVAL_JAC_FLOP_PER_SUB = 35
# Instructions per sub-sample and component of the model loop: 7 VALU and 3
# transcendental (log2, exp2, exp2), for the issue-rate ceiling.
EVAL_VALU_PER_SUB, EVAL_TRANS_PER_SUB = 7, 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=["suite", "c1", "c2", "c3", "c4", "c5", "lines", "cube"], default="suite")
    ap.add_argument("--train-stamps", type=int, default=200_000, help="C5: rendered training stamps")
    ap.add_argument("--epochs", type=int, default=4, help="C5: training epochs")
    ap.add_argument("--mcmc-steps", type=int, default=2000, help="C4: Metropolis steps of the chain run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="target CPU time per oracle sample")
    ap.add_argument("--breakdown", action="store_true", help="print the per-kernel breakdown to stderr")
    ap.add_argument("--calibrate-peaks", action="store_true",
                    help="only run the triad / FMA / transcendental probes and print the measured peaks")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB device buffer three times (reference for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


# ----------------------------------------------------------------- rooflines
def fft_geometry(H, W, K, L):
    """Per-stamp sizes of the convolution: padded pixels, stamp pixels, OTF bytes."""
    Mh, Mw = H + K - 1, W + K - 1
    return Mh * Mw, H * W, L * (L // 2 + 1) * 8


def fft_conv_flops(L, Mh, H):
    """Nominal arithmetic of one channel's FFT convolution at side L (5 N log2 N
    per complex transform of length N, additions and multiplications counted
    separately): row transforms of the Mh padded rows two real rows at a
    time, forward and inverse column transforms of the L/2 + 1 bins, the
    spectrum product, inverse row transforms of the H kept rows."""
    c = 5.0 * L * math.log2(L)
    Lh = L // 2 + 1
    return (Mh + 1) // 2 * c + 2 * Lh * c + 6 * Lh * L + (H + 1) // 2 * c


def kernel_table(stamps, paths, sides, nch, ncomp, S, nimg=None, shared_otf=False, keep_model=False):
    """Algorithmic work per launch of each kernel when every stamp of the
    batch takes part: (bound, units).  stamps: list of (H, W, K); paths and
    sides from the prepared PSF; nch: Jacobian channels per launch; nimg:
    pixels of the distinct observations (shared-image batches); keep_model:
    a plain LM fit of one-component stamps, whose chi^2 passes also write the
    convolved model and whose Jacobian passes evaluate and convolve every
    channel but Ie's (the normal equations take it from that model)."""
    npad = npix = 0
    f2 = dict(pad=0, pix=0, otf=0, n=0, flops=0.0)
    mp = dict(rows=0, cols=0, irows=0, irows_chi2=0, otf=0, pad=0, pix=0, n=0, flops=0.0)
    for (H, W, K), path, L in zip(stamps, paths, sides):
        pad, pix, otf = fft_geometry(H, W, K, max(L, 2))
        npad += pad
        npix += pix
        if shared_otf and (f2["n"] or mp["n"]):
            otf = 0
        Lh = L // 2 + 1
        if path == 2:
            f2["pad"] += pad
            f2["pix"] += pix
            f2["otf"] += otf
            f2["n"] += 1
            f2["flops"] += fft_conv_flops(L, H + K - 1, H)
        elif path == 1:
            Mh = H + K - 1
            mp["rows"] += 4 * pad + 8 * Mh * Lh
            mp["cols"] += 8 * Mh * Lh + 8 * H * Lh
            mp["irows"] += 8 * H * Lh + 4 * pix
            mp["irows_chi2"] += 8 * H * Lh
            mp["otf"] += otf
            mp["pad"] += pad
            mp["pix"] += pix
            mp["n"] += 1
            mp["flops"] += fft_conv_flops(L, Mh, H)
    img = npix if nimg is None else nimg
    dw = 8 * (img if nimg is not None else f2["pix"])      # data + weight read by the fused chi^2
    dw_mp = 8 * (img if nimg is not None else mp["pix"])
    if keep_model:   # the model written beside the chi^2 partials
        dw += 4 * f2["pix"]
        dw_mp += 4 * mp["pix"]
    nconv = nch - 1 if keep_model else nch   # convolved Jacobian channels
    t = {
        "k_eval": ("alu", npad * ncomp * S * S * EVAL_FLOP_PER_SUB),
        "k_eval_jac": ("alu", npad * ncomp * S * S * EVAL_JAC_FLOP_PER_SUB),
        "k_gram": ("hbm", npix * (4 * nch + 8)),
        "k_chi2": ("hbm", 4 * npix + 8 * img),
        # the one-workgroup convolutions move only their definitional bytes
        "k_fft2d": ("hbm", nconv * (4 * f2["pad"] + 4 * f2["pix"]) + f2["otf"]),
        "k_fft2d_chi2": ("hbm", 4 * f2["pad"] + dw + f2["otf"]),
        # the multi-pass kernels: each pass's own reads and writes (spectra
        # included)
        "k_fft_rows": ("hbm", nconv * mp["rows"]),
        "k_fft_cols": ("hbm", nconv * mp["cols"] + mp["otf"]),
        "k_fft_irows": ("hbm", nconv * mp["irows"]),
        "k_fft_rows.chi2": ("hbm", mp["rows"]),
        "k_fft_cols.chi2": ("hbm", mp["cols"] + mp["otf"]),
        "k_fft_irows_chi2": ("hbm", mp["irows_chi2"] + dw_mp),
    }
    stage = dict(
        # step 2 of the Jacobian channels: padded model in, stamp out, OTF once
        convolution=dict(kernels=["k_fft2d", "k_fft_rows", "k_fft_cols", "k_fft_irows"],
                         bytes=nconv * (4 * (f2["pad"] + mp["pad"]) + 4 * (f2["pix"] + mp["pix"])) + f2["otf"] +
                         mp["otf"], flops=nconv * (f2["flops"] + mp["flops"])),
        # steps 2-3 of a model evaluation: padded model, data and weight in,
        # OTF once, only chi^2 out
        convolution_chi2=dict(kernels=["k_fft2d_chi2", "k_fft_rows.chi2", "k_fft_cols.chi2", "k_fft_irows_chi2"],
                              bytes=4 * (f2["pad"] + mp["pad"]) + dw + dw_mp + f2["otf"] + mp["otf"]
                              - (8 * img if nimg is not None else 0), flops=f2["flops"] + mp["flops"]),
        fused_convolution=dict(kernels=["k_fft2d"], bytes=nconv * (4 * f2["pad"] + 4 * f2["pix"]) + f2["otf"],
                               flops=nconv * f2["flops"]),
        fused_convolution_chi2=dict(kernels=["k_fft2d_chi2"], bytes=4 * f2["pad"] + dw + f2["otf"],
                                    flops=f2["flops"]),
        multipass_convolution=dict(kernels=["k_fft_rows", "k_fft_cols", "k_fft_irows"],
                                   bytes=nconv * (4 * mp["pad"] + 4 * mp["pix"]) + mp["otf"],
                                   flops=nconv * mp["flops"]),
    )
    return t, stage, dict(npad=npad, npix=npix, fused_stamps=f2["n"], multipass_stamps=mp["n"])


def roofline(prof, table, peaks, launches_per_call=None):
    """Dominant kernel of the profile and per-kernel figures.  prof: {name:
    (launches, total ms)}; table: {name: (bound, units per launch)}."""
    total = sum(v[1] for v in prof.values())
    stages = {}
    for k, (n, t) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        e = dict(launches=n, ms_total=round(t, 4), us_per_launch=round(t / n * 1e3, 2), share=round(t / total, 4))
        b = table.get(k)
        if b and b[1] > 0:
            per = t / n * 1e-3
            if b[0] == "hbm":
                e.update(bound="hbm", bytes_per_launch=int(b[1]), gbs=round(b[1] / per / 1e9, 1),
                         frac=round(b[1] / per / 1e9 / HBM_PEAK_GBS, 4))
            else:
                e.update(bound="alu", flop_per_launch=int(b[1]), tflops=round(b[1] / per / 1e12, 2),
                         frac=round(b[1] / per / 1e12 / FP32_PEAK_TFLOPS, 4))
        stages[k] = e
    cand = [k for k in prof if table.get(k) and table[k][1] > 0]
    name = max(cand, key=lambda k: prof[k][1])
    n, t = prof[name]
    bound, units = table[name]
    per = t / n * 1e-3
    if bound == "hbm":
        ach = units / per / 1e9
        rl = dict(bound="hbm", kernel=name, achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                  frac=round(ach / HBM_PEAK_GBS, 4), traffic=None)
        if peaks:
            rl["frac_of_measured_triad"] = round(ach / peaks["triad_gbs"], 4)
    else:
        ach = units / per / 1e12
        rl = dict(bound="alu", kernel=name, achieved=round(ach, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                  frac=round(ach / FP32_PEAK_TFLOPS, 4), traffic=None)
        if peaks:
            rl["measured_fp32_fma_unpacked_tflops"] = peaks["fma_tflops"]
            rl["frac_of_unpacked_fma"] = round(ach / peaks["fma_tflops"], 4)
            if name == "k_eval":
                # issue ceilings of the loop's 7 VALU + 3 transcendental
                # instructions per sub-sample at the measured rates (a VALU
                # instruction at half the FMA flop rate): the two pipes
                # overlapped (the larger of the two times) and serial (their sum)
                sub = units / EVAL_FLOP_PER_SUB
                t_valu = sub * EVAL_VALU_PER_SUB * 2 / (peaks["fma_tflops"] * 1e12)
                t_trans = sub * EVAL_TRANS_PER_SUB / (peaks["transcendental_gops"] * 1e9)
                rl["issue_bound_us"] = dict(valu=round(t_valu * 1e6, 2), transcendental=round(t_trans * 1e6, 2),
                                            overlapped=round(max(t_valu, t_trans) * 1e6, 2),
                                            serial=round((t_valu + t_trans) * 1e6, 2))
                rl["frac_of_overlapped_issue_bound"] = round(max(t_valu, t_trans) / per, 4)
    rl["avg_launch_us"] = round(per * 1e6, 2)
    rl["launches_profiled"] = n
    return rl, stages


def stage_fractions(prof, stage, peaks=None):
    """The definitional-byte fractions of steps 2 and 3 (per call of the
    stage: the summed time of its kernels over the calls profiled).  With the
    measured peaks, a convolution stage also gets its arithmetic floor: the
    nominal FFT operations at the unpacked FP32 rate of one operation per lane
    and cycle (half the measured FMA flop rate), and the fraction of 8 TB/s
    the definitional bytes would reach at that floor."""
    out = {}
    for name, st in stage.items():
        ks = [k for k in st["kernels"] if k in prof]
        if not ks or st["bytes"] <= 0:
            continue
        calls = max(prof[k][0] for k in ks)
        t = sum(prof[k][1] for k in ks) / calls * 1e-3
        e = dict(kernels=ks, calls=calls, bytes_per_call=int(st["bytes"]), us_per_call=round(t * 1e6, 2),
                 gbs=round(st["bytes"] / t / 1e9, 1), frac=round(st["bytes"] / t / 1e9 / HBM_PEAK_GBS, 4))
        if peaks and st.get("flops"):
            floor = st["flops"] / (peaks["fma_tflops"] / 2 * 1e12)
            e.update(fft_flops_nominal=int(st["flops"]), alu_floor_us=round(floor * 1e6, 2),
                     frac_of_alu_floor=round(floor / t, 4),
                     hbm_frac_at_alu_floor=round(st["bytes"] / floor / 1e9 / HBM_PEAK_GBS, 4))
        out[name] = e
    return out


# HBM bytes per launch of a dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by the copy calibration: fetch x2, write x1), as
# summarised in profiles/*_hbm_traffic.md.  Valid only while the kernel
# source is the one the counters were taken on (first 16 hex digits of the
# SHA-256 of each listed source).
TRAFFIC = {
    ("c3", "k_eval_jac"): dict(sources={"paper_1101_2254_amd/csrc/k_eval.hip": "9228be28108cf693"}, bytes=2.6091e+09,
                               summary="profiles/c3_batch_hbm_traffic.md"),
    ("c2", "k_eval_jac"): dict(sources={"paper_1101_2254_amd/csrc/k_eval.hip": "9228be28108cf693"}, bytes=1.8807e+07,
                               summary="profiles/c2_fit_hbm_traffic.md"),
    ("c4", "k_eval"): dict(sources={"paper_1101_2254_amd/csrc/k_eval.hip": "9228be28108cf693"}, bytes=3.8620e+08,
                           summary="profiles/c4_likelihood_hbm_traffic.md"),
    ("cube", "k_cube_jac"): dict(sources={"paper_1101_2254_amd/csrc/k_cube.hip": "fa31c6afd1e9783d"}, bytes=2.5859e+09,
                                 summary="profiles/cube_fit_hbm_traffic.md"),
}


def measured_traffic(workload, rl):
    t = TRAFFIC.get((workload, rl.get("kernel")))
    if not t:
        return None
    for src, sha in t["sources"].items():
        try:
            with open(os.path.join(ROOT, src), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest()[:16] != sha:
                    return None
        except OSError:
            return None
    rl["traffic_source"] = t["summary"]
    return round(t["bytes"], 0)


def profile(ctx, fn):
    """Per-kernel HIP-event timing of fn (run once untimed first, so the
    timed run sees warm code objects and caches)."""
    from paper_1101_2254_amd import _lib
    import torch
    fn()
    torch.cuda.synchronize()
    _lib.gf_profile_start(ctx.ptr)
    out = fn()
    torch.cuda.synchronize()
    _lib.gf_profile_stop(ctx.ptr)
    return _lib.gf_profile_read(ctx.ptr), out


def passes(prof):
    """Steps 1-3 passes that a profiled run made: model evaluations plus
    Jacobian evaluations (each over every stamp still fitting)."""
    return prof.get("k_eval", (0, 0))[0], prof.get("k_eval_jac", (0, 0))[0]


# ----------------------------------------------------------------- workloads
def render_observation(torch, ops, ctx, batch, psf, stamps, seed_of, noise):
    """The library's model at the FP32 truth plus seeded numpy noise."""
    dev = ctx.device
    truth = torch.from_numpy(np.concatenate([s.truth for s in stamps]).astype(np.float32)).to(dev)
    m = ops.model(ctx, batch, psf, truth, 5).cpu().numpy().astype(np.float64)
    off = batch.offsets["pix"]
    d = np.empty_like(m)
    w = np.empty_like(m)
    for i, st in enumerate(stamps):
        sl = slice(off[i], off[i] + st.H * st.W)
        dd, ww = noise(m[sl].reshape(st.H, st.W), st, seed_of(i, st))
        d[sl], w[sl] = dd.ravel(), ww.ravel()
    return torch.from_numpy(d.astype(np.float32)).to(dev), torch.from_numpy(w.astype(np.float32)).to(dev)


def run_c3(args, torch, ops, synth, peaks, steps=None, warmup=None):
    """4096 uneven single-Sersic stamps fitted in one gf_fit_lm call (ftol 1e-5)."""
    dev = torch.device("cuda", 0)
    stamps = synth.c3(4096)
    n = len(stamps)
    ctx = ops.Context(0, autotune_cache=TUNE_FILE)
    H = [s.H for s in stamps]
    K = [s.K for s in stamps]
    batch = ops.Batch(ctx, H, H, K, [1] * n)
    taps = torch.from_numpy(np.concatenate([s.psf.astype(np.float32).ravel() for s in stamps])).to(dev)
    psf = ops.Psf(ctx, batch, taps, ops.GF_CONV_AUTO)
    data, weight = render_observation(torch, ops, ctx, batch, psf, stamps, lambda i, st: st.noise_seed,
                                      lambda m, st, seed: synth.add_gaussian_noise(m, st.noise_sigma, seed))
    lo = np.concatenate([synth.bounds(1, s.H, s.W)[0] for s in stamps])
    hi = np.concatenate([synth.bounds(1, s.H, s.W)[1] for s in stamps])
    lo_t, hi_t = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)
    theta0 = torch.from_numpy(np.concatenate([s.start for s in stamps])).to(dev)

    # The active count is read after every iteration: the batch runs as two
    # lanes, so while the host waits on one lane's count the other lane's
    # iteration keeps the device busy, and finished stamps leave the work
    # lists sooner (123 against 127 ms per batch with a read every fourth
    # iteration).
    poll = 1

    def step(**kw):
        o = dict(ftol=1e-5, max_iter=100, poll_every=poll)
        o.update(kw)
        return ops.fit_lm(ctx, batch, psf, data, weight, theta0, lo=lo_t, hi=hi_t, **o)

    K_ = steps if steps is not None else 5
    W = warmup if warmup is not None else 1
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for _ in range(K_):
        recs.append(step(return_device=True)[1])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / K_ * 1e3
    info = ops.lm_info(recs[-1])
    # the first iteration, kernel by kernel: every stamp is active
    prof, _ = profile(ctx, lambda: step(use_graph=0, max_iter=1))
    geo = [(s.H, s.W, s.K) for s in stamps]
    table, stage, sizes = kernel_table(geo, psf.uses_fft, psf.fft_side, 7, 1, 5, keep_model=True)
    rl, kern = roofline(prof, table, peaks)
    pix = np.array([s.H * s.W for s in stamps], dtype=np.float64)
    evals_pix = float(np.sum((info["nfev"] + info["njev"]) * pix))
    res = dict(
        value=round(n / (ms * 1e-3), 2), unit="fits/s", ms_per_step=round(ms, 3), steps=K_, warmup=W,
        mpix_per_s=round(evals_pix / (ms * 1e-3) / 1e6, 2),
        lm=dict(iters_mean=float(info["iters"].mean()), iters_max=int(info["iters"].max()),
                converged=float((info["status"] == 0).mean()), damping_cap=float((info["reason"] == 4).mean()),
                nfev=int(info["nfev"].sum()), njev=int(info["njev"].sum())),
        config=dict(workload="C3: 4096 uneven single-Sersic stamps (32..256 px, Gaussian/Moffat PSF 15..33 px), "
                             "one gf_fit_lm call to chi2 rel tol 1e-5; one step = the whole batch",
                    stamps=n, pixels=int(pix.sum()), oversample=5, poll_every=poll,
                    fused_fft_stamps=sizes["fused_stamps"],
                    multipass_fft_stamps=sizes["multipass_stamps"]),
        roofline=rl, stages=kern, stage_roofline=stage_fractions(prof, stage, peaks),
        roofline_profile="first LM iteration of the batch, kernel by kernel (every stamp active)")
    return res, dict(stamps=stamps, info=info)


def run_c4(args, torch, ops, synth, peaks, steps=None, warmup=None):
    dev = torch.device("cuda", 0)
    base = synth.c4_truth()
    nvec = 1024
    ctx = ops.Context(0)
    batch = ops.Batch(ctx, [256] * nvec, [256] * nvec, [33] * nvec, [1] * nvec, shared=True)
    taps = torch.from_numpy(base.psf.astype(np.float32).ravel()).to(dev)
    psf = ops.Psf(ctx, batch, taps, ops.GF_CONV_AUTO)
    one = ops.Batch(ctx, [256], [256], [33], [1])
    psf1 = ops.Psf(ctx, one, taps, ops.GF_CONV_AUTO)
    m_true = ops.model(ctx, one, psf1, torch.from_numpy(base.truth.astype(np.float32)).to(dev), 5)
    d, w = synth.add_gaussian_noise(m_true.cpu().numpy().astype(np.float64).reshape(256, 256), base.noise_sigma,
                                    base.noise_seed)
    data = torch.from_numpy(d.astype(np.float32).ravel()).to(dev)
    weight = torch.from_numpy(w.astype(np.float32).ravel()).to(dev)
    K = steps if steps is not None else 50
    W = warmup if warmup is not None else 3
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
    ms = (time.perf_counter() - t0) / K * 1e3
    npix = 256 * 256 * nvec
    prof, _ = profile(ctx, lambda: ops.likelihood(ctx, batch, psf, thetas[0], data, weight, 5, work=work, out=out))
    # steps 2 and 3 also through their own entry points
    mp = ops.eval_model(ctx, batch, thetas[0], 5)
    mc = ops.convolve_psf(ctx, batch, psf, mp)

    def sep():
        for _ in range(5):
            ops.convolve_psf(ctx, batch, psf, mp, out=mc)
            ops.chi2(ctx, batch, mc, thetas[0], data, weight)

    sep_prof, _ = profile(ctx, sep)
    del mp, mc
    geo = [(256, 256, 33)] * nvec
    table, stage, sizes = kernel_table(geo, psf.uses_fft, psf.fft_side, 1, 1, 5, nimg=256 * 256, shared_otf=True)
    rl, kern = roofline(prof, table, peaks)
    rl["traffic"] = measured_traffic("c4", rl)
    sr = stage_fractions(prof, stage, peaks)
    sep_stage = {"convolution": stage["convolution"],
                 "chi2": dict(kernels=["k_chi2", "k_pair_final"], bytes=4 * npix + 8 * 256 * 256)}
    for k, v in stage_fractions(sep_prof, sep_stage, peaks).items():
        sr["separate_" + k] = v
    res = dict(
        value=round(npix / (ms * 1e-3) / 1e6, 3), unit="Mpix/s", ms_per_step=round(ms, 4), steps=K, warmup=W,
        config=dict(workload="C4: likelihood batch, 1024 parameter vectors x one 256x256 image, 33x33 Moffat PSF, "
                             "288-point FFT, 5x5 oversampling; one step = steps 1-3 for all vectors",
                    image=[256, 256], psf=33, fft_side=int(psf.fft_side[0]), fft_form=int(psf.uses_fft[0]),
                    vectors=nvec, oversample=5),
        roofline=rl, stages=kern, stage_roofline=sr)
    if args.mcmc_steps > 0:
        res["mcmc"] = run_mcmc(args, torch, ops, synth, ctx, batch, psf, data, weight, thetas[0], base, nvec, npix)
    return res, dict(base=base, thetas_host=synth.c4_vectors(W, nvec), npix=npix)


def run_mcmc(args, torch, ops, synth, ctx, batch, psf, data, weight, theta, base, nvec, npix):
    """Metropolis chains on the likelihood batch: one chain per vector, each
    step = steps 1-3 for all chains."""
    dev = ctx.device
    n_mc = args.mcmc_steps
    scale = torch.from_numpy(np.tile(np.abs(base.truth) * 1e-4 + 1e-6, nvec)).to(dev)
    lo_b, hi_b = synth.bounds(1, 256, 256)
    lo_m = torch.from_numpy(np.tile(lo_b, nvec)).to(dev)
    hi_m = torch.from_numpy(np.tile(hi_b, nvec)).to(dev)
    th_mc = theta.double()
    ops.mcmc_run(ctx, batch, psf, data, weight, th_mc, scale, 10, key=(4004, 1), lo=lo_m, hi=hi_m,
                 keep_samples=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, acc = ops.mcmc_run(ctx, batch, psf, data, weight, th_mc, scale, n_mc, key=(4004, 1), stream=1,
                                lo=lo_m, hi=hi_m, keep_samples=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return dict(chains=nvec, steps=n_mc, ms_per_step=round(t / n_mc * 1e3, 4), mpix_per_s=round(npix * n_mc / t / 1e6, 1),
                accept_rate=round(float(acc.double().mean().item()) / n_mc, 4),
                proposal="theta' = theta + (1e-4 |theta_true| + 1e-6) z, flat prior on the fit bounds")


def run_single(torch, ops, synth, st, ncomp, noise, K_, W, peaks, workload, label):
    """One-image fits (C1, C2): K_ whole fits from the seeded start, timed
    back to back; the result records stay on the device until the end."""
    dev = torch.device("cuda", 0)
    ctx = ops.Context(0, autotune_cache=TUNE_FILE)
    batch = ops.Batch(ctx, [st.H], [st.W], [st.K], [ncomp])
    taps = torch.from_numpy(st.psf.astype(np.float32).ravel()).to(dev)
    psf = ops.Psf(ctx, batch, taps, ops.GF_CONV_AUTO)
    data, weight = render_observation(torch, ops, ctx, batch, psf, [st], lambda i, s: s.noise_seed, noise)
    lo, hi = synth.bounds(ncomp, st.H, st.W)
    lo_t, hi_t = torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev)
    theta0 = torch.from_numpy(st.start).to(dev)

    def step(**kw):
        o = dict(ftol=1e-5, max_iter=100)
        o.update(kw)
        return ops.fit_lm(ctx, batch, psf, data, weight, theta0, lo=lo_t, hi=hi_t, **o)

    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [step(return_device=True)[1] for _ in range(K_)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / K_ * 1e3
    infos = [ops.lm_info(r) for r in recs]
    info = infos[-1]
    if any(int(i["nfev"][0]) != int(info["nfev"][0]) for i in infos):
        raise RuntimeError("fits of the same input took different paths")
    prof, _ = profile(ctx, lambda: step(use_graph=0))
    n_model, n_jac = passes(prof)
    npix = st.H * st.W
    nch = 7 * ncomp
    table, stage, sizes = kernel_table([(st.H, st.W, st.K)], psf.uses_fft, psf.fft_side, nch, ncomp, 5)
    rl, kern = roofline(prof, table, peaks)
    rl["traffic"] = measured_traffic(workload, rl)
    res = dict(
        value=round(1e3 / ms, 3), unit="fits/s", ms_per_step=round(ms, 4), steps=K_, warmup=W,
        mpix_per_s=round((n_model + n_jac) * npix / (ms * 1e-3) / 1e6, 3),
        lm=dict(iters=int(info["iters"][0]), nfev=int(info["nfev"][0]), njev=int(info["njev"][0]),
                status=int(info["status"][0]), reason=int(info["reason"][0]), chi2=float(info["chi2"][0]),
                model_passes=n_model, jacobian_passes=n_jac),
        config=dict(workload=label, image=[st.H, st.W], psf=st.K, fft_side=int(psf.fft_side[0]),
                    fft_form=int(psf.uses_fft[0]), params=7 * ncomp + 1, oversample=5),
        roofline=rl, stages=kern, stage_roofline=stage_fractions(prof, stage, peaks),
        counting="mpix_per_s = (model passes + Jacobian passes the fit ran) x stamp pixels / time per fit")
    return res


def run_c2(args, torch, ops, synth, peaks, steps=None, warmup=None):
    st = synth.c2()
    noise = lambda m, s, seed: synth.add_poisson_read_noise(m, s.meta["read_noise"], s.meta["gain"], seed)
    res = run_single(torch, ops, synth, st, 2, noise, steps if steps is not None else 100,
                     warmup if warmup is not None else 5, peaks, "c2",
                     "C2: one 512x512 image, Sersic bulge + exponential disk, 65x65 Moffat PSF (beta=3, FWHM=3 px), "
                     "576-point FFT convolution, 5x5 oversampling, 15-parameter LM fit to chi2 rel tol 1e-5; "
                     "one step = one whole fit")
    return res, dict(st=st, nfev=res["lm"]["nfev"], njev=res["lm"]["njev"], iters=res["lm"]["iters"])


def run_c1(args, torch, ops, synth, peaks, steps=None, warmup=None):
    st = synth.c1()
    noise = lambda m, s, seed: synth.add_gaussian_noise(m, s.noise_sigma, seed)
    res = run_single(torch, ops, synth, st, 1, noise, steps if steps is not None else 200,
                     warmup if warmup is not None else 5, peaks, "c1",
                     "C1: one 64x64 stamp, one Sersic component (n=2.5, Re=8), 15x15 Gaussian PSF, noise 0.02, "
                     "8-parameter LM fit from a +-20% start to chi2 rel tol 1e-5; one step = one whole fit")
    res["roofline"] = dict(res["roofline"], note="latency-bound single small stamp: reported for completeness")
    return res, dict(st=st)


# Proposal network work per stamp (multiply-adds of the four 3x3 stride-2
# convolutions at 128 x 128 input plus the two dense layers), times two for
# FLOPs; a training step costs about three forward passes.
CNN_MAC_PER_STAMP = (64 * 64 * 32 * 9 * 1 + 32 * 32 * 32 * 9 * 32 + 16 * 16 * 64 * 9 * 32 + 8 * 8 * 64 * 9 * 64
                     + 4096 * 256 + 256 * 8)


def run_c5(args, torch, ops, synth, peaks, steps=None, warmup=None):
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
        o = dict(ftol=1e-5, max_iter=100)
        o.update(kw)
        return ops.fit_lm(ctx, ev.batch, ev.psf, data, weight, start, lo=lo_t, hi=hi_t, **o)

    def step_cnn(**kw):
        return fit(net.predict(data).reshape(-1).contiguous(), **kw)

    def step_default():
        return fit(PR.moments_guess(ctx, ev.batch, data))

    K_ = steps if steps is not None else 5
    W = warmup if warmup is not None else 1
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
    ic, idf = infos["cnn"], infos["default"]
    rel = (ic["chi2"] - idf["chi2"]) / idf["chi2"]
    gemm_ms = tprof.get("k_gemm_bf16", (0, 0.0))[1]
    step_ms = sum(v[1] for v in tprof.values())
    train_flop = 3 * 2 * CNN_MAC_PER_STAMP * 256
    result = dict(
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
    # roofline of the first LM iteration of the network-seeded fit (every
    # stamp active)
    prof1, _ = profile(ctx, lambda: fit(net.predict(data).reshape(-1).contiguous(), use_graph=0, max_iter=1))
    table, stage, _ = kernel_table([(side, side, int(k)) for k in ev.batch.K], ev.psf.uses_fft, ev.psf.fft_side, 7, 1, 5,
                                   keep_model=True)
    rl, kern = roofline(prof1, table, peaks)
    result.update(steps=K_, warmup=W, roofline=rl, stages=kern, stage_roofline=stage_fractions(prof1, stage, peaks),
                  roofline_profile="first LM iteration of the network-seeded fit, kernel by kernel")
    return result, dict(info=ic, nfev=int(ic["nfev"].sum()), njev=int(ic["njev"].sum()))


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


def run_lines(args, torch, ops, synth, peaks, steps=None, warmup=None):
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

    K = steps if steps is not None else 20
    W = warmup if warmup is not None else 3
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
        value=round(n / (ms * 1e-3), 2), unit="fits/s", ms_per_step=round(ms, 4),
        mpix_per_s=round(chan_evals / (ms * 1e-3) / 1e6, 2),
        lm=dict(iters_mean=float(info["iters"].mean()), iters_max=int(info["iters"].max()),
                converged=float((info["status"] == 0).mean()), nfev=int(info["nfev"].sum()),
                njev=int(info["njev"].sum())),
        config=dict(workload="lines: 65536 spectra of 256..2048 channels with 1..3 Gaussian emission lines and a "
                             "continuum, 7..21-tap Gaussian LSF, 5x sub-sampling, one gf_line_fit_lm call to chi2 "
                             "rel tol 1e-5; one step = the whole batch",
                    spectra=n, channels=nch, oversample=S))
    rl, kern = roofline(prof, {"k_line_lm": ("alu", flops)}, peaks)
    result.update(steps=K, warmup=W, roofline=rl, stages=kern)
    return result, dict(spectra=spectra, info=info, data=d, weight=w)


# Algorithmic FP32 operations per (spatial sub-sample, spectral sub-sample,
# padded channel) of the cube kernels (an FMA counts two, exp2 one): the model
# 6 (offset, square, scale, exp2, FMA), the 11 derivative channels 37.
CUBE_EVAL_FLOP, CUBE_JAC_FLOP = 6, 37


def run_cube(args, torch, ops, synth, peaks, steps=None, warmup=None):
    """256 integral-field cubes (32..64 spaxels square, 64 channels, PSF 9..15
    px, 7-tap LSF) of rotating disk galaxies fitted by one gf_cube_fit_lm call
    to chi^2 rel tol 1e-5 (S = 5, Sv = 3)."""
    dev = torch.device("cuda", 0)
    cubes = synth.cube_batch(256)
    n, Nc, Kl = len(cubes), cubes[0].Nc, cubes[0].Kl
    S, Sv = 5, 3
    ctx = ops.Context(0, autotune_cache=TUNE_FILE)
    cb = ops.CubeBatch(ctx, [c.H for c in cubes], [c.W for c in cubes], [c.K for c in cubes], Nc, Kl)
    cb.set_kernels(torch.from_numpy(np.concatenate([c.psf.astype(np.float32).ravel() for c in cubes])).to(dev),
                   torch.from_numpy(np.concatenate([c.lsf.astype(np.float32) for c in cubes])).to(dev))
    truth = torch.from_numpy(np.concatenate([c.truth for c in cubes])).to(dev)
    m = ops.cube_model(ctx, cb, truth, S, Sv).cpu().numpy().astype(np.float64)
    off = cb.offsets["vox"]
    d = np.empty_like(m)
    w = np.empty_like(m)
    for i, c in enumerate(cubes):
        sl = slice(off[i], off[i + 1])
        d[sl], w[sl] = synth.add_gaussian_noise(m[sl], c.noise_sigma, c.noise_seed)
    data = torch.from_numpy(d.astype(np.float32)).to(dev)
    weight = torch.from_numpy(w.astype(np.float32)).to(dev)
    lo = torch.from_numpy(np.concatenate([synth.cube_bounds(c.H, c.W, Nc)[0] for c in cubes])).to(dev)
    hi = torch.from_numpy(np.concatenate([synth.cube_bounds(c.H, c.W, Nc)[1] for c in cubes])).to(dev)
    start = torch.from_numpy(np.concatenate([c.start for c in cubes])).to(dev)

    def step(**kw):
        o = dict(ftol=1e-5, max_iter=100, oversample=S)
        o.update(kw)
        return ops.cube_fit_lm(ctx, cb, data, weight, start, Sv, lo=lo, hi=hi, return_device=True, **o)

    K_ = steps if steps is not None else 5
    W = warmup if warmup is not None else 1
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K_):
        th, res = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / K_ * 1e3
    info = ops.lm_info(res)
    # the first iteration kernel by kernel (every cube active): start model,
    # Jacobian, trial model
    prof, _ = profile(ctx, lambda: step(max_iter=1))
    Mc = Nc + Kl - 1
    samples = sum((c.H + c.K - 1) * (c.W + c.K - 1) for c in cubes) * S * S * Mc * Sv
    lsf_bytes = sum((c.H + c.K - 1) * (c.W + c.K - 1) for c in cubes) * (Mc + Nc) * 4
    table = {"k_cube_jac": ("alu", samples * CUBE_JAC_FLOP), "k_cube_eval": ("alu", samples * CUBE_EVAL_FLOP),
             # start model, Jacobian (every block but Ie's, which the kept model gives), trial model
             "k_cube_lsf": ("hbm", lsf_bytes * (1 + 10 + 1) / 3)}
    rl, kern = roofline(prof, table, peaks)
    rl["traffic"] = measured_traffic("cube", rl)
    vox = np.array([Nc * c.H * c.W for c in cubes], dtype=np.float64)
    passes_vox = float(np.sum((info["nfev"] + info["njev"]) * vox))
    res_d = dict(
        value=round(n / (ms * 1e-3), 2), unit="fits/s", ms_per_step=round(ms, 3), steps=K_, warmup=W,
        mvox_per_s=round(passes_vox / (ms * 1e-3) / 1e6, 2),
        lm=dict(iters_mean=float(info["iters"].mean()), iters_max=int(info["iters"].max()),
                converged=float((info["status"] == 0).mean()), nfev=int(info["nfev"].sum()),
                njev=int(info["njev"].sum())),
        counting="mvox_per_s = sum over cubes of (nfev + njev) x voxels / time per batch",
        config=dict(workload="cube: 256 integral-field cubes of rotating disk galaxies (32..64 spaxels square, 64 "
                             "channels, Gaussian/Moffat PSF 9..15 px, 7-tap Gaussian LSF), 12-parameter LM fit of "
                             "each by one gf_cube_fit_lm call to chi2 rel tol 1e-5, 5x5 spatial and 3 spectral "
                             "sub-samples; one step = the whole batch",
                    cubes=n, channels=Nc, voxels=int(vox.sum()), oversample=S, oversample_v=Sv),
        roofline=rl, stages=kern, roofline_profile="first LM iteration of the batch, kernel by kernel")
    return res_d, dict(cubes=cubes, info=info, data=d, weight=w, off=off, S=S, Sv=Sv)


def cpu_baseline_cube(extra, seconds):
    """The cube oracle (numpy FP64, one thread): one LM iteration (Jacobian,
    solve, trial model) on the batch's first cube of the smallest size, scaled
    to the batch by padded spatial samples and by the GPU fit's iterations per
    cube (extrapolated, labelled so)."""
    from oracle import cube_ref as CR
    import synth
    cubes, info, d, w, off = extra["cubes"], extra["info"], extra["data"], extra["weight"], extra["off"]
    S, Sv = extra["S"], extra["Sv"]
    i = min(range(len(cubes)), key=lambda k: cubes[k].H * cubes[k].W)
    c = cubes[i]
    lo, hi = synth.cube_bounds(c.H, c.W, c.Nc)
    dd = d[off[i]:off[i + 1]].astype(np.float32).astype(np.float64).reshape(c.Nc, c.H, c.W)
    ww = w[off[i]:off[i + 1]].astype(np.float32).astype(np.float64).reshape(c.Nc, c.H, c.W)
    t0 = time.perf_counter()
    CR.fit_lm(c.start, c.psf.astype(np.float32).astype(np.float64), c.lsf.astype(np.float32).astype(np.float64),
              dd, ww, S, Sv, lo=lo, hi=hi, max_iter=1)
    t1 = time.perf_counter() - t0
    pad = lambda cc: (cc.H + cc.K - 1) * (cc.W + cc.K - 1)
    total = sum(t1 * pad(cc) / pad(c) * max(int(info["iters"][k]), 1) for k, cc in enumerate(cubes))
    return dict(value=round(len(cubes) / total, 4), unit="fits/s", cores=1, kind="oracle",
                sample=f"extrapolated: one numpy FP64 oracle LM iteration on cube {i} ({c.H}x{c.W}x{c.Nc}, "
                       f"{t1:.1f} s on one thread), scaled by padded spaxels and by each cube's GPU iterations")


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




# --------------------------------------------------------------- CPU baselines
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_native():
    """The oracle rebuilt for this host (-O3 -march=native, same rounding)."""
    from oracle import gfo
    gfo.use_native(os.path.join(ROOT, "bench_out", "oracle_native"))
    return gfo


def _threads(gfo, n):
    gfo.set_threads(n)
    return gfo.get_threads()


def cpu_baseline_c3(extra, seconds):
    """Stratified sample: one stamp per size class, the oracle's whole LM fit
    (ftol 1e-5) on its own rendering of that stamp on all host cores; one
    iteration per size on one thread, times the all-core fit's iterations.
    Both extrapolated to the batch's stamps per size (labelled so)."""
    import synth
    gfo = oracle_native()
    stamps = extra["stamps"]
    ncores = os.cpu_count() or 1
    per_size = {}
    for N in synth.C3_SIZES:
        idx = [i for i, st in enumerate(stamps) if st.H == N]
        if idx:
            per_size[N] = (stamps[idx[0]], len(idx))
    tot_all = tot_one = 0.0
    used = []
    for N, (st, count) in per_size.items():
        psf = st.psf.astype(np.float32).astype(np.float64)
        m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64), psf, 5)
        d, w = synth.add_gaussian_noise(m, st.noise_sigma, st.noise_seed)
        d, w = d.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64)
        lo, hi = synth.bounds(1, st.H, st.W)
        _threads(gfo, ncores)
        t0 = time.perf_counter()
        _, info = gfo.fit_lm(st.start, psf, d, w, 5, lo=lo, hi=hi, ftol=1e-5, max_iter=100)
        t_fit = time.perf_counter() - t0
        _threads(gfo, 1)
        t0 = time.perf_counter()
        gfo.fit_lm(st.start, psf, d, w, 5, lo=lo, hi=hi, ftol=1e-5, max_iter=1)
        t_it = time.perf_counter() - t0
        tot_all += t_fit * count
        tot_one += t_it * max(info["iters"], 1) * count
        used.append(f"{N}px:{info['iters']}it,{t_fit * 1e3:.0f}ms/{ncores}t,{t_it * 1e3:.0f}ms/it/1t")
    n = len(stamps)
    return dict(value=round(n / tot_all, 3), unit="fits/s", cores=ncores, kind="oracle",
                value_1thread=round(n / tot_one, 4), cores_1thread=1, cpu=cpu_model(), build="gcc -O3 -march=native",
                sample="extrapolated: per stamp size one whole oracle LM fit to ftol 1e-5 on its own rendering "
                       f"(all {ncores} cores) and one iteration on one thread times that fit's iterations, scaled "
                       "by the batch's stamps per size (" + "; ".join(used) + ")")


def cpu_baseline_c4(extra, seconds):
    """The oracle on its own rendering of the same image: steps 1-3 for as
    many of a step's parameter vectors as fit in the time budget, on all
    cores and on one thread."""
    import synth
    gfo = oracle_native()
    base = extra["base"]
    psf = base.psf.astype(np.float32).astype(np.float64)
    m_true = gfo.model(256, 256, base.truth.astype(np.float32).astype(np.float64), psf, 5)
    d, w = synth.add_gaussian_noise(m_true, base.noise_sigma, base.noise_seed)
    d, w = d.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64)
    th = extra["thetas_host"].astype(np.float32).astype(np.float64)
    out = {}
    for label, nt, budget in (("all", os.cpu_count() or 1, seconds / 2), ("one", 1, seconds / 2)):
        _threads(gfo, nt)
        t0 = time.perf_counter()
        n = 0
        while (time.perf_counter() - t0 < budget or n == 0) and n < th.shape[0]:
            gfo.chi2(d, w, gfo.model(256, 256, th[n], psf, 5))
            n += 1
        out[label] = (n, time.perf_counter() - t0, gfo.get_threads())
    n, t, c = out["all"]
    n1, t1, _ = out["one"]
    ctx_fft = cpu_fft_context(gfo, "c4", extra, seconds / 2)
    return dict(value=round(n * 65536 / t / 1e6, 5), unit="Mpix/s", cores=c, kind="oracle", fft_context=ctx_fft,
                value_1thread=round(n1 * 65536 / t1 / 1e6, 6), cores_1thread=1, cpu=cpu_model(),
                build="gcc -O3 -march=native",
                sample=f"FP64 oracle eval + direct convolution + chi2 of {n} (all cores, {t:.1f} s) and {n1} (one "
                       f"thread, {t1:.1f} s) of a step's parameter vectors on its own rendering of the image")


def _fft_valid(pads, otf, L, K, H, W, workers):
    """'Valid' convolution of padded FP64 images (..., Mh, Mw) with a PSF
    given by its L x L OTF, through scipy's FFT on `workers` threads."""
    import scipy.fft as sf
    spec = sf.rfft2(pads, s=(L, L), workers=workers)
    full = sf.irfft2(spec * otf, s=(L, L), workers=workers)
    return full[..., K - 1:K - 1 + H, K - 1:K - 1 + W]


def cpu_fft_context(gfo, kind, extra, seconds):
    """Context for the oracle figures: the same steps with the convolution
    through scipy's FFT (FP64, all host cores) instead of the direct sum.
    kind "c4": steps 1-3 per parameter vector, Mpix/s; kind "c2": one
    Jacobian pass (14 derivative channels on the padded grid, their
    convolutions, the normal equations) times the GPU fit's passes, fits/s.
    Checked against the direct convolution on the first image."""
    import scipy.fft as sf
    nt = os.cpu_count() or 1
    _threads(gfo, nt)
    if kind == "c4":
        base = extra["base"]
        H = W = 256
        psf = base.psf.astype(np.float32).astype(np.float64)
        K = psf.shape[0]
        L = 288
        otf = sf.rfft2(psf, s=(L, L), workers=nt)
        th = extra["thetas_host"].astype(np.float32).astype(np.float64)
        import synth
        m_true = gfo.model(H, W, base.truth.astype(np.float32).astype(np.float64), psf, 5)
        d, w = synth.add_gaussian_noise(m_true, base.noise_sigma, base.noise_seed)
        pad0 = gfo.eval_padded(H, W, K, th[0], 5)
        ref = gfo.conv_valid(pad0, psf)
        got = _fft_valid(pad0, otf, L, K, H, W, nt)
        assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
        t0 = time.perf_counter()
        n = 0
        while (time.perf_counter() - t0 < seconds or n == 0) and n < th.shape[0]:
            m = _fft_valid(gfo.eval_padded(H, W, K, th[n], 5), otf, L, K, H, W, nt) + th[n][-1]
            float(np.sum(w * (d - m) ** 2))
            n += 1
        t = time.perf_counter() - t0
        return dict(value=round(n * H * W / t / 1e6, 4), unit="Mpix/s", cores=gfo.get_threads(),
                    sample=f"{n} vectors in {t:.1f} s: oracle evaluation (C, all cores) + scipy.fft convolution "
                           f"(FP64, {nt} workers) + chi2")
    st = extra["st"]
    psf = st.psf.astype(np.float32).astype(np.float64)
    K = psf.shape[0]
    H, W = st.H, st.W
    L = 576
    otf = sf.rfft2(psf, s=(L, L), workers=nt)
    theta = st.start.astype(np.float64)
    t0 = time.perf_counter()
    dp = gfo.dpadded(H, W, K, theta, 5)                       # (P - 1, Mh, Mw)
    J = _fft_valid(dp, otf, L, K, H, W, nt).reshape(dp.shape[0], -1)
    A = J @ J.T
    t = time.perf_counter() - t0
    ref = gfo.conv_valid(dp[0], psf)
    assert np.abs(J[0].reshape(H, W) - ref).max() <= 1e-9 * np.abs(ref).max()
    passes = max(int(extra.get("njev", 1)) + 1, 1)
    per_fit = t * passes
    return dict(value=round(1.0 / per_fit, 5), unit="fits/s", cores=gfo.get_threads(),
                sample=f"one Jacobian pass ({dp.shape[0]} channels: oracle derivatives on all cores, scipy.fft "
                       f"convolutions with {nt} workers, normal equations) in {t:.2f} s, times the GPU fit's "
                       f"{passes} evaluation passes")


def cpu_baseline_single(extra, seconds, ncomp, label, whole_fits):
    """C1 and C2: whole oracle fits (C1) or the first LM iterations (C2, one
    fit takes minutes) on its own rendering of the same observation."""
    import synth
    gfo = oracle_native()
    st = extra["st"]
    psf = st.psf.astype(np.float32).astype(np.float64)
    m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64), psf, 5)
    if ncomp == 2:
        d, w = synth.add_poisson_read_noise(m, st.meta["read_noise"], st.meta["gain"], st.noise_seed)
    else:
        d, w = synth.add_gaussian_noise(m, st.noise_sigma, st.noise_seed)
    d, w = d.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64)
    lo, hi = synth.bounds(ncomp, st.H, st.W)
    out = {}
    for lab, nt in (("all", os.cpu_count() or 1), ("one", 1)):
        _threads(gfo, nt)
        if whole_fits:
            t0 = time.perf_counter()
            _, info = gfo.fit_lm(st.start, psf, d, w, 5, lo=lo, hi=hi, ftol=1e-5, max_iter=100)
            out[lab] = (time.perf_counter() - t0, info["iters"], "whole fit")
        else:
            t0 = time.perf_counter()
            _, info = gfo.fit_lm(st.start, psf, d, w, 5, lo=lo, hi=hi, ftol=1e-5, max_iter=1)
            t_it = time.perf_counter() - t0
            out[lab] = (t_it * extra["iters"], extra["iters"], "one iteration x the GPU fit's iterations")
    (t, it, how), (t1, _, _) = out["all"], out["one"]
    extra_ctx = {"fft_context": cpu_fft_context(gfo, "c2", extra, seconds)} if ncomp == 2 else {}
    return dict(value=round(1.0 / t, 5), unit="fits/s", ms_per_fit=round(t * 1e3, 2), cores=os.cpu_count() or 1,
                **extra_ctx,
                kind="oracle", value_1thread=round(1.0 / t1, 6), ms_per_fit_1thread=round(t1 * 1e3, 2),
                cores_1thread=1, cpu=cpu_model(), build="gcc -O3 -march=native",
                sample=f"{label}: FP64 oracle LM ({how}; {it} iterations) on its own rendering of the same "
                       "observation, direct convolution")


def calibrate_peaks(ctx):
    from paper_1101_2254_amd import _lib
    ctx.bind_stream()
    out = dict(triad_gbs=round(_lib.gf_probe(ctx.ptr, 0, 1 << 28, 10), 1),
               fma_tflops=round(_lib.gf_probe(ctx.ptr, 1, 4096, 5), 2),
               transcendental_gops=round(_lib.gf_probe(ctx.ptr, 2, 2048, 5), 1))
    out["triad_frac_of_8tbs"] = round(out["triad_gbs"] / HBM_PEAK_GBS, 4)
    return out


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



RUNNERS = dict(c1=run_c1, c2=run_c2, c3=run_c3, c4=run_c4, c5=run_c5, lines=run_lines, cube=run_cube)
DATA = dict(c5="synthetic (seeded; stamps rendered by the library from on-device Philox4x64-10 prior draws and "
                "noise)",
            lines="synthetic (seeded; spectra rendered by the library, noise from numpy PCG64)",
            cube="synthetic (seeded; cubes rendered by the library, noise from numpy PCG64)")


def cpu_for(name, extra, seconds):
    if name == "c3":
        return cpu_baseline_c3(extra, seconds)
    if name == "c4":
        return cpu_baseline_c4(extra, seconds)
    if name == "c2":
        return cpu_baseline_single(extra, seconds, 2, "C2", False)
    if name == "c1":
        return cpu_baseline_single(extra, seconds, 1, "C1", True)
    if name == "c5":
        return cpu_baseline_c5(extra, seconds)
    if name == "cube":
        return cpu_baseline_cube(extra, seconds)
    return cpu_baseline_lines(extra, seconds)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py: the library runs on one GPU; --gpus {max(args.gpus, world)} is not supported "
              "(the hot path shards as described in the design notes, but only the one-GPU kernel is built)",
              file=sys.stderr)
        sys.exit(2)
    os.makedirs(os.path.dirname(TUNE_FILE), exist_ok=True)
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
    os.makedirs(os.path.dirname(TUNE_FILE), exist_ok=True)
    pctx = ops.Context(0)
    peaks = calibrate_peaks(pctx)
    pctx.close()
    if args.calibrate_peaks:
        print(json.dumps(peaks))
        return
    head = "c3" if args.workload == "suite" else args.workload
    log(f"workload {head}")
    res, extra = RUNNERS[head](args, torch, ops, synth, peaks, args.steps, args.warmup)
    log(f"{head}: {res['value']} {res['unit']}, {res['ms_per_step']} ms/step")
    if args.breakdown:
        print(json.dumps(res.get("stages", {}), indent=1), file=sys.stderr)
    if res.get("roofline") and res["roofline"].get("traffic") is None:
        res["roofline"]["traffic"] = measured_traffic(head, res["roofline"])
    out = dict(metric=METRIC, value=res.pop("value"), unit=res.pop("unit"), n_gpus=1, steps=res.pop("steps"),
               warmup=res.pop("warmup"), ms_per_step=res.pop("ms_per_step"), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32",
               data=DATA.get(head, "synthetic (seeded; Sersic stamps rendered by the library, noise from numpy PCG64)"),
               config=res.pop("config"), roofline=res.pop("roofline", None))
    out.update(res)
    nested = {}
    if args.workload == "suite":
        for name in ("c4", "c2", "c1", "cube"):
            log(f"workload {name}")
            r, e = RUNNERS[name](args, torch, ops, synth, peaks)
            log(f"{name}: {r['value']} {r['unit']}, {r['ms_per_step']} ms/step")
            nested[name] = (r, e)
            out[name] = r
    out["peaks_measured"] = peaks
    if not args.no_cpu:
        log("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_for(head, extra, args.cpu_seconds)
        for name, (r, e) in nested.items():
            r["cpu_baseline"] = cpu_for(name, e, args.cpu_seconds / 2)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
