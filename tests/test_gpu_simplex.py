"""GPU parity of the batched downhill simplex against the FP64 reference.

Tolerance of a chi^2 value away from the minimum: with the model image
accurate to eps_m = 2e-6 (relative L2, FP32 evaluation and FFT), the
Cauchy-Schwarz bound |d chi^2| <= 2 sqrt(chi^2) |sqrt(w) dm| + |sqrt(w) dm|^2
gives |d chi^2| <= 1e-5 chi^2 + 2 eps_m sqrt(chi^2) |sqrt(w) m|; at a good fit
the first term dominates (the 1e-5 relative target), at the trial points of
a search the second can (a point at chi^2/N = 2.7 with a 7e-7 model error
differs by 1.3e-5 relative).

Both sides evaluate the same sequence of points until a comparison decides
between two chi^2 values closer than 1e-4 (relative), beyond which either
branch is valid.  Up to the first such comparison the chi^2 traces must
agree to the bound above; at the end both must have converged to the same
minimum value (1e-4 relative) from that start."""
import numpy as np
import pytest
import torch

import synth
from oracle import gfo
from oracle import simplex_ref as NM
from paper_1101_2254_amd import ops
from tests.gpu_common import GpuBatch, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("gpu simplex: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def test_simplex_matches_reference(ctx):
    g = synth.rng(2468)
    stamps = [synth.c1()] + [synth.c3_stamp(g, 32, i, 2468) for i in range(2)]
    data, weights = [], []
    for i, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64),
                      st.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, 300 + i)
        data.append(d.astype(np.float32))
        weights.append(w.astype(np.float32))
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    start = np.concatenate([st.start for st in stamps])
    step = np.concatenate([np.where(np.arange(8) < 2, 0.1 * st.truth[3], 0.05 * np.abs(st.start) + 1e-3)
                           for st in stamps])
    lo = np.concatenate([synth.bounds(1, st.H, st.W)[0] for st in stamps])
    hi = np.concatenate([synth.bounds(1, st.H, st.W)[1] for st in stamps])
    cap = 4000
    print("gpu simplex fit", flush=True)
    th, info, trace = ops.fit_simplex(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(start, torch.float64),
                                      to_dev(step, torch.float64), lo=to_dev(lo, torch.float64),
                                      hi=to_dev(hi, torch.float64), max_iter=3000, ftol=1e-8, trace_cap=cap)
    th = th.cpu().numpy()
    trace = trace.cpu().numpy()
    for s, st in enumerate(stamps):
        print(f"reference stamp {s}", flush=True)
        p64 = gb.psf64(s)
        d64, w64 = gb.d32[s].astype(np.float64), gb.w32[s].astype(np.float64)
        mnorm = []

        def fun(x):
            mm = gfo.model(st.H, st.W, x, p64, 5)
            mnorm.append(float(np.sqrt(np.sum(w64 * mm * mm))))
            return gfo.chi2(d64, w64, mm)
        o = 8 * s
        x, fb, it, nfev, ok, rtrace, margins = NM.minimize(fun, start[o:o + 8], step[o:o + 8], lo[o:o + 8],
                                                           hi[o:o + 8], ftol=1e-8, max_iter=3000)
        first_tie = min([n for n, m in margins if m < 1e-4], default=nfev)
        n_cmp = min(first_tie, cap, int(info["nfev"][s]))
        assert n_cmp >= 50, (s, first_tie)
        ref = np.array(rtrace[:n_cmp])
        tol = 1e-5 * ref + 2 * 2e-6 * np.sqrt(ref) * np.array(mnorm[:n_cmp])
        assert np.all(np.abs(trace[s, :n_cmp] - ref) <= tol), (s, np.max(np.abs(trace[s, :n_cmp] - ref) / tol))
        assert ok and info["status"][s] == 0, (s, info[s])
        ng = int(info["nfev"][s])
        if ng <= cap:
            assert info["chi2"][s] == np.min(trace[s, :ng])
        c_ret = fun(th[o:o + 8])
        assert abs(info["chi2"][s] - c_ret) <= 1e-5 * c_ret + 4e-6 * np.sqrt(c_ret) * mnorm[-1]
        assert info["chi2"][s] <= ref[-1]
        if first_tie >= nfev:   # no near tie: the very same path
            assert info["chi2"][s] == pytest.approx(fb, rel=1e-5)
            assert int(info["nfev"][s]) == nfev
            np.testing.assert_allclose(th[o:o + 8], x, rtol=1e-9, atol=1e-12)
