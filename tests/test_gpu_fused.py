"""The fused chi^2 path (the inverse-row FFT pass reducing chi^2 per output
row pair, direct-path stamps through the chi^2 kernel at their own slots) on
ragged shapes: odd heights (a last row pair with one row), a one-row stamp,
widths that are not multiples of anything, and FFT and direct stamps in one
batch.  Checked against the separate entry points, the FP64 oracle, and
single-stamp fits."""
import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import ops
from tests.gpu_common import keep_fft_forms, GpuBatch, to_dev

pytestmark = pytest.mark.gpu

# (H, W, K): K <= 7 takes the direct path, the rest the FFT path
SHAPES = [(33, 47, 9), (17, 64, 15), (1, 40, 5), (65, 31, 21), (50, 77, 25), (63, 63, 7), (2, 3, 3), (41, 40, 11)]


@pytest.fixture(scope="module")
def ctx():
    print("gpu fused chi2: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    keep_fft_forms(c)   # the fit test compares a stamp alone with the same stamp in the batch, bit for bit
    yield c
    torch.cuda.synchronize()
    c.close()


def _stamps(seed):
    g = synth.rng(seed)
    out = []
    for i, (H, W, K) in enumerate(SHAPES):
        re = max(1.0, 0.15 * min(H, W))
        t = np.array([W / 2 + g.uniform(-0.4, 0.4), H / 2 + g.uniform(-0.4, 0.4), g.uniform(0.8, 2.0), re,
                      g.uniform(1.0, 4.0), g.uniform(0.5, 1.0), g.uniform(0, np.pi), g.uniform(0.0, 0.05)])
        st = t.copy()
        st[2] *= 1.1
        st[3] *= 0.9
        st[4] *= 1.1
        out.append(synth.Stamp(H, W, synth.gaussian_psf(K, 1.2), t, st, 0.02, seed * 100 + i))
    return out


def _observed(gfo, stamps):
    data, weights = [], []
    for s in stamps:
        m = gfo.model(s.H, s.W, s.truth.astype(np.float32).astype(np.float64), s.psf.astype(np.float32).astype(np.float64),
                      5)
        d, w = synth.add_gaussian_noise(m, 0.02, s.noise_seed)
        data.append(d)
        weights.append(w)
    return data, weights


def test_fused_likelihood_ragged(ctx, gfo):
    stamps = _stamps(31)
    data, weights = _observed(gfo, stamps)
    th = [s.start for s in stamps]
    gb = GpuBatch(ctx, stamps, thetas=th, data=data, weights=weights)
    uses = list(gb.psf.uses_fft)
    assert any(uses) and not all(uses)
    print("fused likelihood on ragged shapes", flush=True)
    pairs = ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5)
    chi = ops.pairs_to_f64(pairs).cpu().numpy()
    mp = ops.eval_model(ctx, gb.batch, gb.theta, 5)
    mc = ops.convolve_psf(ctx, gb.batch, gb.psf, mp)
    p2, _ = ops.chi2(ctx, gb.batch, mc, gb.theta, gb.data, gb.weight)
    np.testing.assert_allclose(chi, ops.pairs_to_f64(p2).cpu().numpy(), rtol=5e-8, atol=0)
    for s, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, gb.th64(s), gb.psf64(s), 5)
        ref = gfo.chi2(gb.d32[s].astype(np.float64), gb.w32[s].astype(np.float64), m)
        wm = np.sqrt(np.sum(gb.w32[s] * m * m))
        assert abs(chi[s] - ref) <= 1e-5 * ref + 2 * 2e-6 * np.sqrt(ref) * wm, (s, st.H, st.W, st.K, chi[s], ref)
    assert torch.equal(pairs, ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5))


@pytest.mark.parametrize("spec", [0, 1])
def test_fused_fit_ragged_batch_and_alone(ctx, gfo, spec):
    stamps = _stamps(32)
    data, weights = _observed(gfo, stamps)
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    lo = np.concatenate([synth.bounds(1, s.H, s.W)[0] for s in stamps])
    hi = np.concatenate([synth.bounds(1, s.H, s.W)[1] for s in stamps])
    start = np.concatenate([s.start for s in stamps])
    print(f"fit of the ragged batch, speculate={spec}", flush=True)
    th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(start, torch.float64),
                          lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=1e-5, speculate=spec)
    th = th.cpu().numpy()
    assert np.all(np.isfinite(th)) and np.all(info["iters"] >= 1)
    po = gb.batch.offsets["par"]
    for s, st in enumerate(stamps):
        one = GpuBatch(ctx, [st], data=[data[s]], weights=[weights[s]])
        l, h = synth.bounds(1, st.H, st.W)
        t1, i1 = ops.fit_lm(ctx, one.batch, one.psf, one.data, one.weight, to_dev(st.start, torch.float64),
                            lo=to_dev(l, torch.float64), hi=to_dev(h, torch.float64), ftol=1e-5, speculate=spec)
        np.testing.assert_array_equal(t1.cpu().numpy(), th[po[s]:po[s] + 8], err_msg=str(s))
        assert i1["chi2"][0] == info["chi2"][s] and i1["iters"][0] == info["iters"][s], s
    # the reported chi^2 is the oracle's at the returned parameters
    for s, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, th[po[s]:po[s] + 8], gb.psf64(s), 5)
        ref = gfo.chi2(gb.d32[s].astype(np.float64), gb.w32[s].astype(np.float64), m)
        wm = np.sqrt(np.sum(gb.w32[s] * m * m))
        assert abs(info["chi2"][s] - ref) <= 1e-5 * ref + 2 * 2e-6 * np.sqrt(ref) * wm + 1e-9, (s, info["chi2"][s], ref)


def test_concurrent_fft_forms_same_bits(gfo):
    """A batch with stamps on both FFT forms: the one-workgroup launches run
    on the context's side stream beside the multi-pass ones, in eager calls
    and inside the captured LM iteration.  With timing records on, both run
    on the calling stream; the two orders give the same bits."""
    from paper_1101_2254_amd import _lib as L
    stamps = _stamps(33)
    data, weights = _observed(gfo, stamps)
    lo = np.concatenate([synth.bounds(1, s.H, s.W)[0] for s in stamps])
    hi = np.concatenate([synth.bounds(1, s.H, s.W)[1] for s in stamps])
    start = np.concatenate([s.start for s in stamps])
    out = []
    for timed in (False, True):
        c = ops.Context(0)
        keep_fft_forms(c)
        probe = GpuBatch(c, stamps, data=data, weights=weights)
        sides = sorted({int(s) for u, s in zip(probe.psf.uses_fft, probe.psf.fft_side) if u})
        L.gf_tune_form_set(c.ptr, sides[0], 1)      # the smallest FFT side on the multi-pass form
        gb = GpuBatch(c, stamps, thetas=[s.start for s in stamps], data=data, weights=weights)
        assert {1, 2} <= set(int(u) for u in gb.psf.uses_fft), list(gb.psf.uses_fft)
        print(f"both FFT forms, timing records {'on' if timed else 'off'}", flush=True)
        if timed:
            L.gf_profile_start(c.ptr)
        pairs = ops.likelihood(c, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5)
        mc = ops.convolve_psf(c, gb.batch, gb.psf, ops.eval_model(c, gb.batch, gb.theta, 5))
        th, info = ops.fit_lm(c, gb.batch, gb.psf, gb.data, gb.weight, to_dev(start, torch.float64),
                              lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=1e-8)
        torch.cuda.synchronize()
        if timed:
            L.gf_profile_stop(c.ptr)
        out.append((pairs.cpu(), mc.cpu(), th.cpu(), info))
        c.close()
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][2], out[1][2])
    for k in ("chi2", "iters", "nfev"):
        np.testing.assert_array_equal(out[0][3][k], out[1][3][k])
