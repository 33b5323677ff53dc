"""GPU parity of the two forms of the FFT convolution against the FP64 oracle's
direct "valid" convolution, at every FFT side the benchmarked workloads reach
and at every side of the one-workgroup form.

* one-workgroup form (GF_CONV_FFT_FUSED): every side class it is built for
  (8 ... 192), a square stamp whose padded side is exactly L and a ragged
  one (odd H, W < L), one and three channels;
* multi-pass form (GF_CONV_FFT_MULTIPASS): the sides of the single-image fit
  (576), the uneven batch and the learned-proposal stamps (48 ... 288), one
  and seven channels (seven = a Jacobian's channels per component);
* the chi^2 epilogue and the adjoint correlation of both forms;
* both forms on one mixed batch.

Model images relative L2 <= 1e-5 per stamp and channel (the tolerance of
the model image)."""
import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import _lib as L
from paper_1101_2254_amd import ops
from tests.gpu_common import GpuBatch, rel_l2, to_dev

pytestmark = pytest.mark.gpu

FUSED_SIDES = [8, 10, 12, 16, 18, 20, 24, 30, 32, 36, 40, 48, 50, 54, 60, 64, 72, 80, 90, 96, 100, 108, 120, 128,
               144, 150, 160, 162, 180, 192]
# sides reached by the uneven batch (stamps 32..256 with PSFs 15..33), the
# learned-proposal stamps (128 with 15..33) and the single-image fit (576)
WORKLOAD_SIDES = [48, 50, 54, 60, 64, 72, 80, 90, 96, 120, 128, 144, 150, 160, 216, 240, 270, 288]


@pytest.fixture(scope="module")
def ctx():
    print("gpu fft forms: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _shapes_for(L_side):
    """(H, W, K) of a square stamp with padded side exactly L and a ragged
    one (odd sides, padded grid smaller than L in both directions, but with
    the same FFT side)."""
    K = 15 if L_side >= 24 else 3
    H = L_side - K + 1
    Hr = H - 1 if (H - 1) % 2 == 1 else H - 2
    Wr = max(1, H - 5) | 1
    return [(H, H, K), (Hr, Wr, K)]


def _conv_case(ctx, gfo, shapes, mode, n_ch, seed):
    g = synth.rng(seed)
    stamps = []
    for (H, W, K) in shapes:
        th = np.array([W / 2, H / 2, 1.0, 3.0, 2.0, 0.7, 0.4, 0.0])
        stamps.append(synth.Stamp(H, W, synth.random_psf(K, int(g.integers(1000))), th, th))
    gb = GpuBatch(ctx, stamps, mode=mode)
    ins = [(g.standard_normal((n_ch, st.H + st.K - 1, st.W + st.K - 1)) + 2.0).astype(np.float32) for st in stamps]
    flat = to_dev(np.concatenate([x.ravel() for x in ins]))
    out = gb.split_pix(ops.convolve_psf(ctx, gb.batch, gb.psf, flat, n_ch), n_ch)
    for s, st in enumerate(stamps):
        for c in range(n_ch):
            ref = gfo.conv_valid(ins[s][c].astype(np.float64), gb.psf64(s))
            got = out[s][c] if n_ch > 1 else out[s]
            err = rel_l2(got, ref)
            assert err <= 1e-5, f"stamp {s} ch {c} {st.H}x{st.W} K={st.K} L={gb.psf.fft_side[s]}: {err:.2e}"
    return gb


@pytest.mark.parametrize("side", FUSED_SIDES)
def test_fused_conv_every_side(ctx, gfo, side):
    print(f"fused conv L={side}", flush=True)
    for n_ch in (1, 3):
        gb = _conv_case(ctx, gfo, _shapes_for(side), ops.GF_CONV_FFT_FUSED, n_ch, 1000 + side)
        assert list(gb.psf.uses_fft) == [2, 2] and list(gb.psf.fft_side) == [side, side]


@pytest.mark.parametrize("side", WORKLOAD_SIDES)
def test_multipass_conv_workload_sides(ctx, gfo, side):
    print(f"multi-pass conv L={side}", flush=True)
    for n_ch in (1, 7):
        gb = _conv_case(ctx, gfo, _shapes_for(side), ops.GF_CONV_FFT_MULTIPASS, n_ch, 2000 + side)
        assert list(gb.psf.uses_fft) == [1, 1] and list(gb.psf.fft_side) == [side, side]


def test_multipass_conv_576_seven_channels_sampled(ctx, gfo):
    """The single-image fit's side (512 x 512, 65 x 65 PSF) with the seven
    channels of one component's Jacobian: 200 pixels per channel against
    the direct sum, one by one."""
    g = synth.rng(576)
    psf = synth.moffat_psf(65, 3.0, 3.0)
    th = np.array([256.0, 256.0, 1.0, 3.0, 2.0, 0.7, 0.4, 0.0])
    st = synth.Stamp(512, 512, psf, th, th)
    gb = GpuBatch(ctx, [st], mode=ops.GF_CONV_FFT_MULTIPASS)
    assert gb.psf.fft_side[0] == 576
    ins = (g.standard_normal((7, 576, 576)) + 2.0).astype(np.float32)
    out = gb.split_pix(ops.convolve_psf(ctx, gb.batch, gb.psf, to_dev(ins.ravel()), 7), 7)[0]
    p64 = gb.psf64(0)
    for c in range(7):
        pts = [(int(g.integers(0, 512)), int(g.integers(0, 512))) for _ in range(200)] + [(0, 0), (511, 511)]
        got = np.array([out[c][i, j] for i, j in pts])
        ref = np.array([gfo.conv_valid_pixel(ins[c].astype(np.float64), p64, i, j) for i, j in pts])
        assert rel_l2(got, ref) <= 1e-5, c


def test_both_forms_in_one_batch(ctx, gfo):
    """Automatic choice on a batch whose sides straddle the one-workgroup
    limit: small stamps take that form, large ones the multi-pass form, and
    all convolve correctly in one call (three channels)."""
    shapes = [(40, 40, 15), (120, 100, 21), (178, 178, 15), (200, 190, 17), (64, 64, 33), (250, 250, 21)]
    gb = _conv_case(ctx, gfo, shapes, ops.GF_CONV_AUTO, 3, 77)
    paths = list(gb.psf.uses_fft)
    sides = list(gb.psf.fft_side)
    for p, s in zip(paths, sides):
        assert p == (2 if s <= 160 else 1), (paths, sides)
    assert 1 in paths and 2 in paths


def test_fused_side_limit_is_refused(ctx):
    b = ops.Batch(ctx, [200], [200], [15], [1])
    taps = to_dev(np.full(225, 1.0 / 225, np.float32))
    try:
        L.gf_psf_prepare(ctx.ptr, b.ptr, int(taps.data_ptr()), L.GF_CONV_FFT_FUSED)
        raised = False
    except L.GfError as e:
        raised = e.status == L.GF_ESHAPE
    assert raised


def _observed(gfo, stamps, seed):
    data, weights = [], []
    for s, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64),
                      st.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, seed + s)
        data.append(d)
        weights.append(w)
    return data, weights


@pytest.mark.parametrize("mode", [ops.GF_CONV_FFT_FUSED, ops.GF_CONV_FFT_MULTIPASS])
def test_chi2_epilogue_both_forms(ctx, gfo, mode):
    """Steps 1-3 in one call (the chi^2 formed where the model rows leave
    on-chip memory) on uneven stamps up to 128 px, away from the truth,
    against the oracle's chi^2 of its own model."""
    g = synth.rng(4321)
    stamps = [synth.c3_stamp(g, int(g.choice([32, 48, 64, 96, 128])), i, 4321) for i in range(8)]
    data, weights = _observed(gfo, stamps, 300)
    thetas = [st.start for st in stamps]
    gb = GpuBatch(ctx, stamps, thetas=thetas, data=data, weights=weights, mode=mode)
    assert all(u == (2 if mode == ops.GF_CONV_FFT_FUSED else 1) for u in gb.psf.uses_fft)
    print(f"chi2 epilogue mode {mode}", flush=True)
    chi = ops.pairs_to_f64(ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5)).cpu().numpy()
    for s, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, gb.th64(s), gb.psf64(s), 5)
        ref = gfo.chi2(gb.d32[s], gb.w32[s], m)
        # away from the minimum the FP32 model error enters through the cross
        # term: |d chi2| <= 1e-5 chi2 + 2 eps sqrt(chi2) ||sqrt(w) m||
        wm = np.sqrt(np.sum(gb.w32[s] * m * m))
        assert abs(chi[s] - ref) <= 1e-5 * ref + 2 * 2e-6 * np.sqrt(ref) * wm, (s, chi[s], ref)
    # the separate calls agree with the fused chi^2 (same model values,
    # reduced per output row pair instead of per pixel chunk)
    mp = ops.eval_model(ctx, gb.batch, gb.theta, 5)
    mc = ops.convolve_psf(ctx, gb.batch, gb.psf, mp)
    p2, _ = ops.chi2(ctx, gb.batch, mc, gb.theta, gb.data, gb.weight)
    np.testing.assert_allclose(chi, ops.pairs_to_f64(p2).cpu().numpy(), rtol=5e-8, atol=0)
    assert torch.equal(ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5),
                       ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5))


@pytest.mark.parametrize("mode", [ops.GF_CONV_FFT_FUSED, ops.GF_CONV_FFT_MULTIPASS])
def test_adjoint_both_forms(ctx, gfo, mode):
    """d chi^2 / d theta through the adjoint correlation of each form, on an
    80 x 80 stamp with a 33 x 33 PSF (side 112 -> 120), against the oracle's
    analytic gradient."""
    th = np.array([40.3, 39.6, 1.5, 6.0, 2.5, 0.6, 0.8, 0.01])
    st = synth.Stamp(80, 80, synth.moffat_psf(33, 3.0, 3.0), th, th * np.array([1.002, 0.998, 1.1, 0.9, 1.1, 1.05,
                                                                                     1.02, 1.0]))
    data, weights = _observed(gfo, [st], 91)
    gb = GpuBatch(ctx, [st], thetas=[st.start], data=data, weights=weights, mode=mode)
    mp = ops.eval_model(ctx, gb.batch, gb.theta, 5)
    m = ops.convolve_psf(ctx, gb.batch, gb.psf, mp)
    _, resid = ops.chi2(ctx, gb.batch, m, gb.theta, gb.data, gb.weight, want_resid=True)
    g = ops.jacobian_adjoint(ctx, gb.batch, gb.psf, gb.theta, resid, gb.weight, -2.0, 5).cpu().numpy()
    ref = gfo.grad_chi2(gb.th64(0), gb.psf64(0), gb.d32[0].astype(np.float64), gb.w32[0].astype(np.float64), 5)
    assert np.abs(g - ref).max() <= 1e-4 * np.abs(ref).max(), (g, ref)


def test_restricted_lists_keep_both_forms(ctx, gfo):
    """LM fits on a batch mixing both FFT forms and the direct sum, with the
    work lists restricted to the unfinished stamps at every halving
    (poll_every = 1, several restrictions in a row) and never (poll_every
    large): the same bits for every stamp."""
    g = synth.rng(2468)
    stamps = [synth.c3_stamp(g, N, i, 2468) for i, N in enumerate([32, 48, 64, 96, 128, 192, 256, 32, 64, 128])]
    small = synth.Stamp(40, 40, synth.gaussian_psf(7, 1.2), stamps[0].truth.copy(), stamps[0].start.copy())
    small.truth[0:2] = small.start[0:2] = [20.2, 19.7]
    small.truth[3] = small.start[3] = 5.0
    stamps.append(small)
    data, weights = _observed(gfo, stamps, 1234)
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    paths = set(gb.psf.uses_fft)
    assert paths == {0, 1, 2}, paths
    lo = to_dev(np.concatenate([synth.bounds(1, st.H, st.W)[0] for st in stamps]), torch.float64)
    hi = to_dev(np.concatenate([synth.bounds(1, st.H, st.W)[1] for st in stamps]), torch.float64)
    start = to_dev(np.concatenate([st.start for st in stamps]), torch.float64)
    def fits():
        out = []
        for pe in (1, 1000):
            th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-8,
                                  poll_every=pe, speculate=0)
            out.append((th.cpu().numpy(), info))
        return out

    sides = sorted({int(s) for s, u in zip(gb.psf.fft_side, gb.psf.uses_fft) if u == 2})
    keep = {s: L.gf_tune_min_active_get(ctx.ptr, s) for s in sides}
    try:
        # the one-workgroup stamps keep their form to the end: the same bits
        for s in sides:
            L.gf_tune_min_active_set(ctx.ptr, s, 0)
        out = fits()
        assert len(set(out[1][1]["iters"])) > 2    # stamps finish at different iterations
        np.testing.assert_array_equal(out[0][0], out[1][0])
        for k in ("chi2", "iters", "nfev", "status"):
            np.testing.assert_array_equal(out[0][1][k], out[1][1][k])
        # every stamp moves to the multi-pass form at the first restriction:
        # the same minima (both forms compute the same convolution to
        # rounding)
        for s in sides:
            L.gf_tune_min_active_set(ctx.ptr, s, 1 << 20)
        out2 = fits()
        np.testing.assert_allclose(out2[0][1]["chi2"], out2[1][1]["chi2"], rtol=1e-5)
        np.testing.assert_allclose(out2[0][1]["chi2"], out[1][1]["chi2"], rtol=1e-5)
    finally:
        for s, v in keep.items():
            L.gf_tune_min_active_set(ctx.ptr, s, v)
