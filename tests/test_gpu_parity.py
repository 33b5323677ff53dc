"""GPU parity: every entry point of include/gf.h against the FP64 oracle on the
same FP32 inputs.

Tolerances: model images relative L2 <= 1e-5, chi^2 relative <= 1e-5, fitted
parameters |d theta| <= 1e-4 max(|theta|, s) (s = Re for centres, pi for the
position angle compared mod pi, the noise sigma for the sky).  Jacobian
images are held to 1e-4 relative L2 per parameter: each pixel derivative is
a sum of sub-sample terms that largely cancel (the centre derivatives are odd
about the centre), so FP32 rounding of the terms is amplified relative to the
result.
"""
import math

import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import ops
from tests.gpu_common import keep_fft_forms, GpuBatch, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("gpu parity: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    keep_fft_forms(c)
    yield c
    torch.cuda.synchronize()
    c.close()


def _edge_stamps():
    """Stamps at the edges of the parameter box, plus a centre that sits
    exactly on a sub-sample (R = 0 is sampled)."""
    g = synth.rng(4242)
    out = []
    for (N, K, th) in [
        (32, 15, [16.0, 16.0, 2.0, 3.0, 6.0, 0.9, 0.3, 0.02]),      # centre on a sub-sample, cusp
        (48, 17, [23.7, 24.4, 0.7, 12.0, 0.5, 0.2, 2.0, 0.0]),      # Gaussian, very flat
        (64, 21, [31.1, 33.9, 3.0, 2.0, 4.0, 0.05, 1.2, 0.01]),     # q at its lower bound
        (40, 9, [5.3, 34.6, 1.0, 6.0, 1.0, 1.0, 0.0, 0.03]),        # off-centre, round
        (31, 13, [15.2, 14.8, 1.5, 4.0, 10.0, 0.6, -0.7, 0.0]),     # n at its upper bound, odd size
        (37, 11, [18.1, 19.3, 1.5, 4.0, 0.2, 0.6, 3.0, 0.0]),       # n at its lower bound
    ]:
        psf = synth.gaussian_psf(K, 1.7) if K % 4 == 1 else synth.moffat_psf(K, 3.0, 3.0)
        th = np.array(th)
        out.append(synth.Stamp(N, N, psf, th, th.copy(), 0.02, int(g.integers(1 << 30))))
    return out


def _c3_small(n=10, seed=77):
    g = synth.rng(seed)
    return [synth.c3_stamp(g, int(g.choice([32, 48, 64, 96])), i, seed) for i in range(n)]


# --------------------------------------------------------------- step 1
def test_eval_c1(ctx, gfo):
    st = synth.c1()
    gb = GpuBatch(ctx, [st])
    out = ops.eval_model(ctx, gb.batch, gb.theta, 5)
    ref = gfo.eval_padded(st.H, st.W, st.K, gb.th64(0), 5)
    assert rel_l2(gb.split_pad(out)[0], ref) <= 1e-5


def test_eval_uneven_batch_and_edges(ctx, gfo):
    stamps = _c3_small() + _edge_stamps()
    gb = GpuBatch(ctx, stamps)
    out = gb.split_pad(ops.eval_model(ctx, gb.batch, gb.theta, 5))
    for s, st in enumerate(stamps):
        ref = gfo.eval_padded(st.H, st.W, st.K, gb.th64(s), 5)
        assert np.all(np.isfinite(out[s]))
        assert rel_l2(out[s], ref) <= 1e-5, f"stamp {s} ({st.H}x{st.W}, K={st.K}, theta={gb.th32[s]})"


@pytest.mark.parametrize("S", [1, 2, 3, 5, 8])
def test_eval_oversampling(ctx, gfo, S):
    st = synth.c1()
    gb = GpuBatch(ctx, [st])
    out = ops.eval_model(ctx, gb.batch, gb.theta, S)
    ref = gfo.eval_padded(st.H, st.W, st.K, gb.th64(0), S)
    assert rel_l2(gb.split_pad(out)[0], ref) <= 1e-5


def test_eval_two_components_full_size_sampled(ctx, gfo):
    """512x512 bulge + disk with the 65x65 PSF padding (576x576 grid): the
    brightest 15x15 block and 400 random pixels computed one by one."""
    st = synth.c2()
    gb = GpuBatch(ctx, [st])
    out = gb.split_pad(ops.eval_model(ctx, gb.batch, gb.theta, 5))[0]
    c = (st.K - 1) // 2
    g = synth.rng(5)
    cy, cx = int(round(st.truth[1])), int(round(st.truth[0]))
    pts = [(cy + a, cx + b) for a in range(-7, 8) for b in range(-7, 8)]
    pts += [(int(g.integers(-c, st.H + c)), int(g.integers(-c, st.W + c))) for _ in range(400)]
    got = np.array([out[i + c, j + c] for i, j in pts])
    ref = np.array([gfo.pixel(gb.th64(0), 5, i, j) for i, j in pts])
    assert rel_l2(got, ref) <= 1e-5
    assert np.all(np.abs(got - ref) <= 1e-5 * np.abs(ref) + 1e-6 * np.abs(ref).max())


def test_eval_shared_batch_vectors(ctx, gfo):
    """A likelihood batch (one image, many parameter vectors): every vector's
    grid matches its own oracle evaluation."""
    base = synth.c4_truth()
    small = synth.Stamp(64, 64, synth.moffat_psf(33, 3.0, 3.0), base.truth.copy(), base.truth.copy())
    small.truth[0:2] = [32.3, 31.7]
    small.truth[3] = 6.0
    th = np.repeat(small.truth[None, :], 5, 0) * np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    g = synth.rng(9)
    th[:, 2:6] *= 1.0 + 0.05 * g.standard_normal((5, 4))
    gb = GpuBatch(ctx, [small] * 5, thetas=list(th), shared=True)
    out = gb.split_pad(ops.eval_model(ctx, gb.batch, gb.theta, 5))
    for s in range(5):
        ref = gfo.eval_padded(64, 64, 33, gb.th64(s), 5)
        assert rel_l2(out[s], ref) <= 1e-5


# --------------------------------------------------------------- step 2
def _conv_case(ctx, gfo, shapes, mode, n_ch=1, seed=3):
    g = synth.rng(seed)
    stamps = []
    for (H, W, K) in shapes:
        th = np.array([W / 2, H / 2, 1.0, 3.0, 2.0, 0.7, 0.4, 0.0])
        stamps.append(synth.Stamp(H, W, synth.random_psf(K, int(g.integers(1000))), th, th))
    gb = GpuBatch(ctx, stamps, mode=mode)
    ins = []
    for st in stamps:
        Mh, Mw = st.H + st.K - 1, st.W + st.K - 1
        ins.append((g.standard_normal((n_ch, Mh, Mw)) + 2.0).astype(np.float32))
    flat = to_dev(np.concatenate([x.ravel() for x in ins]))
    out = gb.split_pix(ops.convolve_psf(ctx, gb.batch, gb.psf, flat, n_ch), n_ch)
    for s, st in enumerate(stamps):
        for c in range(n_ch):
            ref = gfo.conv_valid(ins[s][c].astype(np.float64), gb.psf64(s))
            got = out[s][c] if n_ch > 1 else out[s]
            assert rel_l2(got, ref) <= 1e-5, f"stamp {s} ch {c} shape {st.H}x{st.W} K={st.K}"
    return gb


def test_conv_fft_sizes(ctx, gfo):
    gb = _conv_case(ctx, gfo, [(64, 64, 15), (48, 40, 21), (96, 96, 33), (32, 32, 17), (50, 77, 25), (16, 16, 3),
                               (128, 100, 19)], ops.GF_CONV_FFT)
    assert all(gb.psf.uses_fft)


def test_conv_direct_sizes(ctx, gfo):
    gb = _conv_case(ctx, gfo, [(64, 64, 15), (20, 70, 9), (33, 65, 5), (17, 16, 1), (70, 20, 41)],
                    ops.GF_CONV_DIRECT)
    assert not any(gb.psf.uses_fft)


@pytest.mark.parametrize("mode", [ops.GF_CONV_FFT, ops.GF_CONV_DIRECT])
def test_conv_channels(ctx, gfo, mode):
    _conv_case(ctx, gfo, [(40, 40, 11), (24, 30, 7)], mode, n_ch=3, seed=11)


def test_conv_full_size_c2_sampled(ctx, gfo):
    """512x512 with the 65x65 Moffat PSF on a 576-point FFT: the oracle's own
    padded model grid (FP32) convolved on the GPU; 300 output pixels checked
    against the direct sum, computed one by one."""
    st = synth.c2()
    gb = GpuBatch(ctx, [st], mode=ops.GF_CONV_FFT)
    assert gb.psf.fft_side[0] == 576
    mp_host = gfo.eval_padded(st.H, st.W, st.K, gb.th64(0), 5).astype(np.float32)
    out = gb.split_pix(ops.convolve_psf(ctx, gb.batch, gb.psf, to_dev(mp_host.ravel())))[0]
    mp64 = mp_host.astype(np.float64)
    g = synth.rng(8)
    cy, cx = int(round(st.truth[1])), int(round(st.truth[0]))
    pts = [(cy + a, cx + b) for a in range(-5, 6) for b in range(-5, 6)]
    pts += [(int(g.integers(0, st.H)), int(g.integers(0, st.W))) for _ in range(300)]
    pts += [(0, 0), (0, st.W - 1), (st.H - 1, 0), (st.H - 1, st.W - 1)]
    got = np.array([out[i, j] for i, j in pts])
    ref = np.array([gfo.conv_valid_pixel(mp64, gb.psf64(0), i, j) for i, j in pts])
    assert rel_l2(got, ref) <= 1e-5


def test_conv_largest_side_sampled(ctx, gfo):
    """The largest FFT side the library takes: a 1920 x 1920 stamp with the
    largest PSF (129 x 129) pads to 2048 x 2048.  A seeded grid of uniform
    values in [0, 1) is convolved on the GPU (multi-pass FFT); the centre,
    the corners and 200 random output pixels are checked against the
    oracle's direct sum, computed one by one."""
    N, K = 1920, 129
    psf = synth.moffat_psf(K, 40.0, 3.0)
    st = synth.Stamp(N, N, psf, np.zeros(8), np.zeros(8))
    gb = GpuBatch(ctx, [st], thetas=[np.zeros(8)], mode=ops.GF_CONV_FFT)
    assert gb.psf.fft_side[0] == 2048 and int(gb.psf.uses_fft[0]) == 1
    g = synth.rng(2048)
    mp_host = g.random((N + K - 1, N + K - 1)).astype(np.float32)
    print("convolution at the largest side", flush=True)
    out = gb.split_pix(ops.convolve_psf(ctx, gb.batch, gb.psf, to_dev(mp_host.ravel())))[0]
    mp64 = mp_host.astype(np.float64)
    pts = [(N // 2, N // 2), (0, 0), (0, N - 1), (N - 1, 0), (N - 1, N - 1)]
    pts += [(int(g.integers(0, N)), int(g.integers(0, N))) for _ in range(200)]
    got = np.array([out[i, j] for i, j in pts])
    ref = np.array([gfo.conv_valid_pixel(mp64, gb.psf64(0), i, j) for i, j in pts])
    assert rel_l2(got, ref) <= 1e-5, rel_l2(got, ref)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_delta_psf_is_identity_on_gpu(ctx, gfo):
    for mode in (ops.GF_CONV_FFT, ops.GF_CONV_DIRECT):
        K = 9
        psf = np.zeros((K, K))
        psf[4, 4] = 1.0
        th = np.array([11.2, 9.7, 1.0, 3.0, 2.2, 0.6, 0.9, 0.05])
        st = synth.Stamp(21, 19, psf, th, th)
        gb = GpuBatch(ctx, [st], mode=mode)
        mp = ops.eval_model(ctx, gb.batch, gb.theta, 5)
        out = gb.split_pix(ops.convolve_psf(ctx, gb.batch, gb.psf, mp))[0]
        pad = gb.split_pad(mp)[0]
        tol = 0 if mode == ops.GF_CONV_DIRECT else 1e-6 * np.abs(pad).max()
        assert np.abs(out - pad[4:4 + 21, 4:4 + 19]).max() <= tol


# --------------------------------------------------------------- step 3
def _observed(gfo, stamps, thetas, seed=0):
    data, weights = [], []
    for s, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, thetas[s], st.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, seed + s)
        data.append(d)
        weights.append(w)
    return data, weights


def test_chi2_and_residual(ctx, gfo):
    stamps = [synth.c1()] + _c3_small(6, seed=91)
    th = [st.truth.astype(np.float32).astype(np.float64) for st in stamps]
    data, weights = _observed(gfo, stamps, th, 100)
    weights[1][:5, :] = 0.0  # masked rows
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    mp = ops.eval_model(ctx, gb.batch, gb.theta, 5)
    m = ops.convolve_psf(ctx, gb.batch, gb.psf, mp)
    pairs, resid = ops.chi2(ctx, gb.batch, m, gb.theta, gb.data, gb.weight, want_resid=True)
    chi = ops.pairs_to_f64(pairs).cpu().numpy()
    ms = gb.split_pix(m)
    rs = gb.split_pix(resid)
    for s, st in enumerate(stamps):
        # the same FP32 model: chi^2 as an exact-ish FP64 sum
        mm = ms[s].astype(np.float64) + np.float64(np.float32(th[s][-1]))
        ref_same, r_ref = gfo.chi2(gb.d32[s], gb.w32[s], mm, want_resid=True)
        assert chi[s] == pytest.approx(ref_same, rel=1e-6)
        # r = sqrt(w) (d - m): FP32 rounding of d - m is amplified by sqrt(w)
        tol = 4 * np.sqrt(gb.w32[s]) * np.finfo(np.float32).eps * (np.abs(gb.d32[s]) + np.abs(mm)) + 1e-30
        assert np.all(np.abs(rs[s] - r_ref) <= tol)
        # against the oracle's own model
        ref = gfo.chi2(gb.d32[s], gb.w32[s], gfo.model(st.H, st.W, gb.th64(s), gb.psf64(s), 5))
        assert chi[s] == pytest.approx(ref, rel=1e-5)
    # bitwise reproducible
    pairs2, _ = ops.chi2(ctx, gb.batch, m, gb.theta, gb.data, gb.weight)
    assert torch.equal(pairs, pairs2)


def test_likelihood_shared_image(ctx, gfo):
    """The likelihood batch: many vectors against one 256x256 image with the
    33x33 Moffat PSF; three vectors checked against the oracle.  48 vectors
    take the wide FFT launch shape, the 4-vector batch the narrow one."""
    base = synth.c4_truth()
    truth64 = base.truth.astype(np.float32).astype(np.float64)
    m = gfo.model(256, 256, truth64, base.psf.astype(np.float32).astype(np.float64), 5)
    d, w = synth.add_gaussian_noise(m, 0.02, base.noise_seed)
    th = synth.c4_vectors(0, 48)
    gb = GpuBatch(ctx, [base] * 48, thetas=list(th), data=[d], weights=[w], shared=True)
    assert len(gb.psf.uses_fft) == 48
    pairs = ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5)
    chi = ops.pairs_to_f64(pairs).cpu().numpy()
    for s in (0, 7, 47):
        ref = gfo.chi2(gb.d32[0], gb.w32[0], gfo.model(256, 256, gb.th64(s), gb.psf64(0), 5))
        assert chi[s] == pytest.approx(ref, rel=1e-5), s
    # the separate calls give the same chi^2: the fused call reduces the same
    # residuals (same model values) per output row pair instead of per pixel
    # chunk, so the two compensated FP32 sums differ only by their own
    # rounding (a few 1e-9 relative over 65536 terms)
    mp = ops.eval_model(ctx, gb.batch, gb.theta, 5)
    mc = ops.convolve_psf(ctx, gb.batch, gb.psf, mp)
    p2, _ = ops.chi2(ctx, gb.batch, mc, gb.theta, gb.data, gb.weight)
    np.testing.assert_allclose(chi, ops.pairs_to_f64(p2).cpu().numpy(), rtol=5e-8, atol=0)
    # and the fused call is bitwise reproducible
    assert torch.equal(pairs, ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5))
    # a small batch of the same vectors (narrow launch shape) agrees
    gs = GpuBatch(ctx, [base] * 4, thetas=list(th[[0, 7, 13, 47]]), data=[d], weights=[w], shared=True)
    chi_s = ops.pairs_to_f64(ops.likelihood(ctx, gs.batch, gs.psf, gs.theta, gs.data, gs.weight, 5)).cpu().numpy()
    np.testing.assert_allclose(chi_s, chi[[0, 7, 13, 47]], rtol=1e-6)


def test_model_entry_point(ctx, gfo):
    stamps = [synth.c1()] + _c3_small(3, seed=5)
    gb = GpuBatch(ctx, stamps)
    out = gb.split_pix(ops.model(ctx, gb.batch, gb.psf, gb.theta, 5))
    for s, st in enumerate(stamps):
        ref = gfo.model(st.H, st.W, gb.th64(s), gb.psf64(s), 5)
        assert rel_l2(out[s], ref) <= 1e-5


# ---------------------------------------------------------- derivatives
@pytest.mark.parametrize("mode", [ops.GF_CONV_DIRECT, ops.GF_CONV_FFT])
def test_jacobian_full(ctx, gfo, mode):
    th1 = np.array([12.3, 11.6, 1.0, 3.0, 2.5, 0.7, 0.5, 0.01])
    th2 = np.array([15.7, 16.2, 1.0, 2.0, 3.5, 0.8, 0.3, 16.1, 15.9, 0.3, 6.0, 1.0, 0.5, 1.9, 0.02])
    stamps = [synth.Stamp(24, 24, synth.gaussian_psf(7, 1.3), th1, th1),
              synth.Stamp(32, 32, synth.moffat_psf(9, 3.0, 3.0), th2, th2)]
    for st in stamps:
        gb = GpuBatch(ctx, [st], mode=mode)
        J = ops.jacobian_full(ctx, gb.batch, gb.psf, gb.theta, 5).cpu().numpy()
        P = st.truth.size
        J = J[:P * st.H * st.W].reshape(P, st.H, st.W)
        ref = gfo.jacobian(st.H, st.W, gb.th64(0), gb.psf64(0), 5)
        for p in range(P):
            assert rel_l2(J[p], ref[p]) <= 1e-4, f"parameter {p}"


def test_adjoint_gradient(ctx, gfo):
    """d chi^2 / d theta from the adjoint kernels against the oracle's
    analytic gradient, away from the minimum."""
    for mode in (ops.GF_CONV_DIRECT, ops.GF_CONV_FFT):
        st = synth.c1()
        th = st.truth.astype(np.float32).astype(np.float64)
        data, weights = _observed(gfo, [st], [th], 7)
        off = (st.start.astype(np.float32)).astype(np.float64)
        gb = GpuBatch(ctx, [st], thetas=[off], data=data, weights=weights, mode=mode)
        mp = ops.eval_model(ctx, gb.batch, gb.theta, 5)
        m = ops.convolve_psf(ctx, gb.batch, gb.psf, mp)
        _, resid = ops.chi2(ctx, gb.batch, m, gb.theta, gb.data, gb.weight, want_resid=True)
        g = ops.jacobian_adjoint(ctx, gb.batch, gb.psf, gb.theta, resid, gb.weight, -2.0, 5).cpu().numpy()
        ref = gfo.grad_chi2(gb.th64(0), gb.psf64(0), gb.d32[0].astype(np.float64), gb.w32[0].astype(np.float64), 5)
        assert np.abs(g - ref).max() <= 1e-4 * np.abs(ref).max(), (g, ref)


def test_autograd_functions(ctx, gfo):
    st = synth.c1()
    th = st.truth.astype(np.float32).astype(np.float64)
    data, weights = _observed(gfo, [st], [th], 17)
    gb = GpuBatch(ctx, [st], thetas=[st.start], data=data, weights=weights)
    theta = gb.theta.clone().requires_grad_(True)
    chi = ops.Chi2Fn.apply(theta, ctx, gb.batch, gb.psf, gb.data, gb.weight, 5)
    chi.sum().backward()
    ref = gfo.grad_chi2(gb.th64(0), gb.psf64(0), gb.d32[0].astype(np.float64), gb.w32[0].astype(np.float64), 5)
    g = theta.grad.cpu().numpy()
    assert np.abs(g - ref).max() <= 1e-4 * np.abs(ref).max()
    theta2 = gb.theta.clone().requires_grad_(True)
    m = ops.ModelFn.apply(theta2, ctx, gb.batch, gb.psf, 5)
    v = to_dev(synth.rng(2).standard_normal(st.H * st.W))
    (m * v).sum().backward()
    J = gfo.jacobian(st.H, st.W, gb.th64(0), gb.psf64(0), 5).reshape(8, -1)
    ref2 = J @ v.cpu().numpy().astype(np.float64)
    assert np.abs(theta2.grad.cpu().numpy() - ref2).max() <= 1e-4 * np.abs(ref2).max()


# -------------------------------------------------------------- LM fit
def _param_close(a, b, ncomp, sigma):
    """|a - b| <= 1e-4 max(|b|, s): s = Re for centres, pi for PA (mod pi), sigma for sky."""
    for k in range(ncomp):
        re = abs(b[7 * k + 3])
        for p in range(7):
            i = 7 * k + p
            if p == 6:
                d = (a[i] - b[i] + math.pi / 2) % math.pi - math.pi / 2
                assert abs(d) <= 1e-4 * math.pi, (i, a[i], b[i])
            else:
                s = re if p in (0, 1) else 0.0
                assert abs(a[i] - b[i]) <= 1e-4 * max(abs(b[i]), s), (i, a[i], b[i])
    assert abs(a[-1] - b[-1]) <= 1e-4 * max(abs(b[-1]), sigma), (a[-1], b[-1])


def test_fit_lm_c1_matches_oracle(ctx, gfo):
    st = synth.c1()
    th = st.truth.astype(np.float32).astype(np.float64)
    data, weights = _observed(gfo, [st], [th], st.noise_seed)
    gb = GpuBatch(ctx, [st], data=data, weights=weights)
    lo, hi = synth.bounds(1, st.H, st.W)
    opts = dict(ftol=1e-12, xtol=1e-10, max_iter=200)
    ref, info = gfo.fit_lm(st.start, gb.psf64(0), gb.d32[0].astype(np.float64), gb.w32[0].astype(np.float64), 5,
                           lo=lo, hi=hi, **opts)
    fit, res = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(st.start, torch.float64),
                          lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), **opts)
    fit = fit.cpu().numpy()
    print("oracle", ref, info)
    print("gpu   ", fit, res)
    _param_close(fit, ref, 1, 0.02)
    assert res["chi2"][0] == pytest.approx(info["chi2"], rel=1e-5)


def test_fit_lm_batch_default_tolerance(ctx, gfo):
    """A batch of uneven stamps (32 to 256 px) fitted at the throughput
    tolerance, ftol = 1e-5, on both sides: every stamp's final chi^2 within
    1e-5 (relative) of the oracle's fit from the same start.  (Parameter
    parity at ftol 1e-12 for the same sizes is in
    test_gpu_workload_parity.py.)"""
    g = synth.rng(123)
    stamps = [synth.c3_stamp(g, N, i, 123) for i, N in enumerate([32, 64, 96, 128, 192, 256])]
    ths = [st.truth.astype(np.float32).astype(np.float64) for st in stamps]
    data, weights = _observed(gfo, stamps, ths, 500)
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    lo = np.concatenate([synth.bounds(1, st.H, st.W)[0] for st in stamps])
    hi = np.concatenate([synth.bounds(1, st.H, st.W)[1] for st in stamps])
    start = np.concatenate([st.start for st in stamps])
    fit, res = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(start, torch.float64),
                          lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=1e-5)
    for s, st in enumerate(stamps):
        l, h = synth.bounds(1, st.H, st.W)
        ref, info = gfo.fit_lm(st.start, gb.psf64(s), gb.d32[s].astype(np.float64), gb.w32[s].astype(np.float64),
                               5, lo=l, hi=h, ftol=1e-5)
        # the oracle converges by ftol; the GPU too, or by the damping cap once
        # its FP32 chi^2 no longer resolves the last decreases, at the same
        # chi^2
        assert info["status"] == 0, (s, info)
        assert res["status"][s] == 0 or res["reason"][s] == 4, (s, res[s])
        assert res["chi2"][s] == pytest.approx(info["chi2"], rel=1e-5), (s, st.H, res[s], info)


def test_fit_lm_two_lanes_default_tolerance(gfo):
    """The six stamps of the test above followed by 594 stamps of 32 px: a
    600-stamp plain fit, which runs as two lanes (the form of the uneven-batch
    benchmark, with the one-workgroup stamps moved to the multi-pass launches
    once few of their bucket remain: a context of its own, with the default
    move thresholds).  The six stamps' final chi^2 within 1e-5 (relative) of
    the oracle's fits from the same start at ftol 1e-5."""
    ctx = ops.Context(0)
    g = synth.rng(123)
    stamps = [synth.c3_stamp(g, N, i, 123) for i, N in enumerate([32, 64, 96, 128, 192, 256])]
    g2 = synth.rng(124)
    stamps += [synth.c3_stamp(g2, 32, 6 + i, 124) for i in range(594)]
    ths = [st.truth.astype(np.float32).astype(np.float64) for st in stamps]
    print("oracle renders 600 stamps", flush=True)
    data, weights = _observed(gfo, stamps, ths, 500)
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    assert {1, 2} <= set(int(u) for u in gb.psf.uses_fft[:6])
    lo = np.concatenate([synth.bounds(1, st.H, st.W)[0] for st in stamps])
    hi = np.concatenate([synth.bounds(1, st.H, st.W)[1] for st in stamps])
    start = np.concatenate([st.start for st in stamps])
    print("two-lane fit of 600 stamps", flush=True)
    fit, res = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(start, torch.float64),
                          lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=1e-5, poll_every=1)
    assert np.all(np.isfinite(fit.cpu().numpy()))
    for s, st in enumerate(stamps[:6]):
        l, h = synth.bounds(1, st.H, st.W)
        print(f"oracle fit of stamp {s} ({st.H} px)", flush=True)
        ref, info = gfo.fit_lm(st.start, gb.psf64(s), gb.d32[s].astype(np.float64), gb.w32[s].astype(np.float64),
                               5, lo=l, hi=h, ftol=1e-5)
        assert info["status"] == 0, (s, info)
        assert res["status"][s] == 0 or res["reason"][s] == 4, (s, res[s])
        assert res["chi2"][s] == pytest.approx(info["chi2"], rel=1e-5), (s, st.H, res[s], info)
    torch.cuda.synchronize()
    ctx.close()


def test_fit_lm_uneven_batch_c3(ctx, gfo):
    """64 stamps with the uneven-size priors (32..256 px, PSF 15..33, Gaussian
    or Moffat) fitted in one call; six small ones checked against the oracle
    from the same start, and one refitted alone must give bitwise the same
    result (a stamp's computation does not depend on the rest of the batch)."""
    g = synth.rng(31337)
    stamps = [synth.c3_stamp(g, int(g.choice(synth.C3_SIZES)), i, 31337) for i in range(64)]
    ths = [st.truth.astype(np.float32).astype(np.float64) for st in stamps]
    data, weights = _observed(gfo, stamps, ths, 900)
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    lo = np.concatenate([synth.bounds(1, st.H, st.W)[0] for st in stamps])
    hi = np.concatenate([synth.bounds(1, st.H, st.W)[1] for st in stamps])
    start = np.concatenate([st.start for st in stamps])
    opts = dict(ftol=1e-12, xtol=1e-10, max_iter=200)
    fit, res = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(start, torch.float64),
                          lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), **opts)
    fit = fit.cpu().numpy()
    assert np.all(np.isfinite(fit))
    assert np.all(res["iters"] >= 1)
    small = [s for s, st in enumerate(stamps) if st.H <= 64][:6]
    for s in small:
        st = stamps[s]
        l, h = synth.bounds(1, st.H, st.W)
        ref, info = gfo.fit_lm(st.start, gb.psf64(s), gb.d32[s].astype(np.float64), gb.w32[s].astype(np.float64),
                               5, lo=l, hi=h, **opts)
        o = gb.batch.offsets["par"][s]
        assert res["chi2"][s] == pytest.approx(info["chi2"], rel=1e-5), s
        _param_close(fit[o:o + 8], ref, 1, 0.02)
    # the same stamp alone, in the batch's (non-speculative) mode
    s = small[0]
    one = GpuBatch(ctx, [stamps[s]], data=[data[s]], weights=[weights[s]])
    l, h = synth.bounds(1, stamps[s].H, stamps[s].W)
    f1, r1 = ops.fit_lm(ctx, one.batch, one.psf, one.data, one.weight, to_dev(stamps[s].start, torch.float64),
                        lo=to_dev(l, torch.float64), hi=to_dev(h, torch.float64), speculate=0, **opts)
    o = gb.batch.offsets["par"][s]
    np.testing.assert_array_equal(f1.cpu().numpy(), fit[o:o + 8])
    assert r1["chi2"][0] == res["chi2"][s] and r1["iters"][0] == res["iters"][s]
