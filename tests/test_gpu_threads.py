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
