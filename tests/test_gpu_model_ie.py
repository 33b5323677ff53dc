"""Plain LM fits take the Ie column of a one-component stamp's normal
equations from the convolved model that the accepted trial's chi^2 pass
kept (the model is linear in Ie: dm/dIe = (m - sky) / Ie) and skip that
channel's evaluation and convolution.  A batch mixing one-component stamps
on all three convolution paths (one-workgroup FFT, multi-pass FFT, direct)
with a two-component stamp (which keeps its convolved Ie channels) is fitted
in the plain form and checked against the FP64 oracle's fits from the same
starts, and each stamp fitted alone gives the same bits as in the batch."""
import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import _lib as L
from paper_1101_2254_amd import ops
from tests.gpu_common import keep_fft_forms, GpuBatch, to_dev

pytestmark = pytest.mark.gpu

OPTS = dict(ftol=1e-12, xtol=1e-10, max_iter=200, speculate=0)


def _two_comp(H, K, seed):
    t = np.array([H / 2 + 0.3, H / 2 - 0.2, 0.8, 4.0, 3.0, 0.8, 0.5,
                  H / 2 + 0.3, H / 2 - 0.2, 0.3, 10.0, 1.0, 0.6, 0.9, 0.01])
    st = t.copy()
    st[[2, 3, 9, 10]] *= [1.1, 0.9, 0.9, 1.1]
    return synth.Stamp(H, H, synth.gaussian_psf(K, 1.3), t, st, 0.02, seed, "two components")


def _stamps():
    g = synth.rng(4242)
    out = [synth.c3_stamp(g, N, i, 4242) for i, N in enumerate([32, 64, 48])]
    out[2].psf = synth.gaussian_psf(5, 1.0)    # K = 5: the direct path
    out.append(_two_comp(48, 9, 4243))
    return out


def _observed(gfo, stamps):
    data, weights = [], []
    for s in stamps:
        m = gfo.model(s.H, s.W, s.truth.astype(np.float32).astype(np.float64),
                      s.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, s.noise_seed)
        data.append(d)
        weights.append(w)
    return data, weights


def _bounds(stamps):
    lo = np.concatenate([synth.bounds(s.ncomp, s.H, s.W)[0] for s in stamps])
    hi = np.concatenate([synth.bounds(s.ncomp, s.H, s.W)[1] for s in stamps])
    return to_dev(lo, torch.float64), to_dev(hi, torch.float64)


def _param_close(a, b, ncomp, sigma):
    for k in range(ncomp):
        re = abs(b[7 * k + 3])
        for p in range(7):
            i = 7 * k + p
            if p == 6:
                d = (a[i] - b[i] + np.pi / 2) % np.pi - np.pi / 2
                assert abs(d) <= 1e-4 * np.pi, (i, a[i], b[i])
            else:
                s = re if p in (0, 1) else 0.0
                assert abs(a[i] - b[i]) <= 1e-4 * max(abs(b[i]), s), (i, a[i], b[i])
    assert abs(a[-1] - b[-1]) <= 1e-4 * max(abs(b[-1]), sigma), (a[-1], b[-1])


def test_plain_fit_model_ie_matches_oracle_and_alone(gfo):
    stamps = _stamps()
    data, weights = _observed(gfo, stamps)
    ctx = ops.Context(0)
    keep_fft_forms(ctx)
    probe = GpuBatch(ctx, stamps, data=data, weights=weights)
    L.gf_tune_form_set(ctx.ptr, int(probe.psf.fft_side[1]), 1)   # the 64 px stamp on the multi-pass form
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    assert [int(u) for u in gb.psf.uses_fft[:3]] == [2, 1, 0], list(gb.psf.uses_fft)
    lo, hi = _bounds(stamps)
    start = np.concatenate([s.start for s in stamps])
    print("plain fit of the mixed batch", flush=True)
    fit, res = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(start, torch.float64), lo=lo, hi=hi,
                          **OPTS)
    fit = fit.cpu().numpy()
    po = gb.batch.offsets["par"]
    for s, st in enumerate(stamps):
        l, h = synth.bounds(st.ncomp, st.H, st.W)
        print(f"oracle fit of stamp {s} ({st.H} px, K = {st.K}, {st.ncomp} component(s))", flush=True)
        ref, info = gfo.fit_lm(st.start, gb.psf64(s), gb.d32[s].astype(np.float64), gb.w32[s].astype(np.float64), 5,
                               lo=l, hi=h, ftol=OPTS["ftol"], xtol=OPTS["xtol"], max_iter=OPTS["max_iter"])
        assert res["chi2"][s] == pytest.approx(info["chi2"], rel=1e-5), (s, res[s], info)
        _param_close(fit[po[s]:po[s] + 7 * st.ncomp + 1], ref, st.ncomp, 0.02)
    for s, st in enumerate(stamps):
        print(f"stamp {s} alone", flush=True)
        one = GpuBatch(ctx, [st], data=[data[s]], weights=[weights[s]])
        l, h = _bounds([st])
        t1, i1 = ops.fit_lm(ctx, one.batch, one.psf, one.data, one.weight, to_dev(st.start, torch.float64), lo=l,
                            hi=h, **OPTS)
        np.testing.assert_array_equal(t1.cpu().numpy(), fit[po[s]:po[s] + 7 * st.ncomp + 1], err_msg=str(s))
        assert i1["chi2"][0] == res["chi2"][s] and i1["iters"][0] == res["iters"][s], s
    torch.cuda.synchronize()
    ctx.close()
