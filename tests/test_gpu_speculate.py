"""Speculative LM iterations (the Jacobian images, normal equations and chi^2
of every trial point from one evaluation) against the plain iterations and
the FP64 oracle: the same fits to the parity bar, chi^2 at the returned
parameters equal to the oracle's, rejected trials (forced by a Gauss-Newton
first step) handled by reusing the stored normal equations, and the edge
cases of the start point."""
import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import _lib as L
from paper_1101_2254_amd import ops
from tests.gpu_common import keep_fft_forms, GpuBatch, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("gpu speculate: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    keep_fft_forms(c)
    yield c
    torch.cuda.synchronize()
    c.close()


def _problem(ctx, gfo, stamps):
    data, weights = [], []
    for s in stamps:
        m = gfo.model(s.H, s.W, s.truth.astype(np.float32).astype(np.float64), s.psf.astype(np.float32).astype(np.float64),
                      5)
        d, w = synth.add_gaussian_noise(m, 0.02, s.noise_seed)
        data.append(d)
        weights.append(w)
    gb = GpuBatch(ctx, stamps, data=data, weights=weights)
    lo = np.concatenate([synth.bounds(s.ncomp, s.H, s.W)[0] for s in stamps])
    hi = np.concatenate([synth.bounds(s.ncomp, s.H, s.W)[1] for s in stamps])
    return gb, to_dev(lo, torch.float64), to_dev(hi, torch.float64)


def _check_chi2_at_theta(gfo, gb, th, info):
    po = gb.batch.offsets["par"]
    for s, st in enumerate(gb.stamps):
        m = gfo.model(st.H, st.W, th[po[s]:po[s] + 7 * st.ncomp + 1], gb.psf64(s), 5)
        ref = gfo.chi2(gb.d32[s].astype(np.float64), gb.w32[s].astype(np.float64), m)
        wm = np.sqrt(np.sum(gb.w32[s] * m * m))
        assert abs(info["chi2"][s] - ref) <= 1e-5 * ref + 2 * 2e-6 * np.sqrt(ref) * wm + 1e-9, (s, info["chi2"][s], ref)


def _stamps(seed, n):
    g = synth.rng(seed)
    return [synth.c3_stamp(g, int(N), i, seed * 10 + i) for i, N in enumerate([32, 48, 64, 96, 32, 64][:n])]


@pytest.mark.parametrize("lambda0", [1e-3, 1e-12])
def test_speculative_matches_plain(ctx, gfo, lambda0):
    stamps = _stamps(81, 6)
    gb, lo, hi = _problem(ctx, gfo, stamps)
    start = to_dev(np.concatenate([s.start for s in stamps]), torch.float64)
    out = {}
    for spec in (0, 1):
        print(f"speculate={spec} lambda0={lambda0}", flush=True)
        th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-6,
                              lambda_=lambda0, speculate=spec)
        th = th.cpu().numpy()
        # at this tolerance the FP32 chi^2 may stop resolving the last
        # decreases, so a fit may end by the damping cap at the minimum
        assert np.all(np.isfinite(th)) and np.all((info["status"] == L.GF_OK) | (info["reason"] == 4)), info
        _check_chi2_at_theta(gfo, gb, th, info)
        out[spec] = (th, info)
    (t0, i0), (t1, i1) = out[0], out[1]
    np.testing.assert_allclose(i1["chi2"], i0["chi2"], rtol=1e-5)
    po = gb.batch.offsets["par"]
    for s in range(len(stamps)):
        a, b = t1[po[s]:po[s] + 8], t0[po[s]:po[s] + 8]
        re = abs(b[3])
        for p in range(8):
            if p == 6:
                d = (a[p] - b[p] + np.pi / 2) % np.pi - np.pi / 2
                assert abs(d) <= 1e-3, (s, p, a[p], b[p])
            else:
                sc = re if p in (0, 1) else (0.02 if p == 7 else 0.0)
                assert abs(a[p] - b[p]) <= 1e-3 * max(abs(b[p]), sc), (s, p, a[p], b[p])
    if lambda0 == 1e-12:
        # a Gauss-Newton first step from 20 % off overshoots: rejected trials
        # must have happened (nfev counts the start and every trial, njev the
        # start and every accepted trial but the last)
        assert np.any(i1["nfev"] - i1["njev"] - 1 > 0), i1


def test_speculative_single_stamp_default(ctx, gfo):
    st = synth.c1()
    gb, lo, hi = _problem(ctx, gfo, [st])
    start = to_dev(st.start, torch.float64)
    th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-10)
    th0, info0 = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-10, speculate=0)
    # the default for one stamp is the speculative form: a different chi^2
    # reduction, so the last bits of chi^2 differ from the plain form
    th1, info1 = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-10, speculate=1)
    np.testing.assert_array_equal(th.cpu().numpy(), th1.cpu().numpy())
    assert info["chi2"][0] == info1["chi2"][0]
    assert info["chi2"][0] == pytest.approx(info0["chi2"][0], rel=1e-6)
    ref, rinfo = gfo.fit_lm(st.start, gb.psf64(0), gb.d32[0].astype(np.float64), gb.w32[0].astype(np.float64), 5,
                            lo=lo.cpu().numpy(), hi=hi.cpu().numpy(), ftol=1e-10)
    assert info["chi2"][0] == pytest.approx(rinfo["chi2"], rel=1e-5)
    _check_chi2_at_theta(gfo, gb, th.cpu().numpy(), info)


def test_speculative_edge_cases(ctx, gfo):
    stamps = _stamps(82, 3)
    gb, lo, hi = _problem(ctx, gfo, stamps)
    start = to_dev(np.concatenate([s.start for s in stamps]), torch.float64)
    # zero weights: chi^2 = 0 at the start, no iteration
    w0 = torch.zeros_like(gb.weight)
    th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, w0, start, lo=lo, hi=hi, speculate=1)
    assert np.all(info["reason"] == 3) and np.all(info["iters"] == 0)
    # no iterations: chi^2 of the clipped start
    th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, max_iter=0, speculate=1)
    np.testing.assert_array_equal(th.cpu().numpy(), start.cpu().numpy())
    _check_chi2_at_theta(gfo, gb, th.cpu().numpy(), info)
    assert np.all(info["reason"] == 5)
    # one iteration, then the cap
    th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, max_iter=1, speculate=1)
    assert np.all(info["iters"] == 1)
    _check_chi2_at_theta(gfo, gb, th.cpu().numpy(), info)
    # bad option value
    o = L.gf_lm_opts_default()
    o.speculate = 2
    with pytest.raises(L.GfError):
        L.gf_fit_lm(ctx.ptr, gb.batch.ptr, gb.psf.ptr, int(gb.data.data_ptr()), int(gb.weight.data_ptr()),
                    int(start.data_ptr()), o, int(start.data_ptr()))


def test_speculative_direct_path_stamps(ctx, gfo):
    # small PSFs take the direct convolution: the speculative iterations
    # convolve their Jacobian images on that path too
    g = synth.rng(83)
    stamps = []
    for i, N in enumerate([32, 48, 40]):
        st = synth.c3_stamp(g, N, i, 8300 + i)
        st.psf = synth.gaussian_psf(5, 1.0)
        stamps.append(st)
    gb, lo, hi = _problem(ctx, gfo, stamps)
    assert not any(gb.psf.uses_fft)
    start = to_dev(np.concatenate([s.start for s in stamps]), torch.float64)
    res = {}
    for spec in (0, 1):
        print(f"direct-path stamps, speculate={spec}", flush=True)
        th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-6,
                              speculate=spec)
        th = th.cpu().numpy()
        assert np.all(np.isfinite(th)) and np.all((info["status"] == L.GF_OK) | (info["reason"] == 4)), info
        _check_chi2_at_theta(gfo, gb, th, info)
        res[spec] = info
    np.testing.assert_allclose(res[1]["chi2"], res[0]["chi2"], rtol=1e-5)


def test_speculative_free_mask(ctx, gfo):
    # fixed parameters (n, q and PA held) stay at the start in both forms and
    # the fits reach the same chi^2
    stamps = _stamps(84, 3)
    gb, lo, hi = _problem(ctx, gfo, stamps)
    st0 = np.concatenate([s.start for s in stamps])
    start = to_dev(st0, torch.float64)
    free = np.concatenate([[1, 1, 1, 1, 0, 0, 0, 1] for _ in stamps]).astype(np.uint8)
    out = {}
    for spec in (0, 1):
        print(f"free mask, speculate={spec}", flush=True)
        th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-6,
                              free=to_dev(free, torch.uint8), speculate=spec)
        th = th.cpu().numpy()
        np.testing.assert_array_equal(th[free == 0], np.clip(st0, lo.cpu().numpy(), hi.cpu().numpy())[free == 0])
        _check_chi2_at_theta(gfo, gb, th, info)
        out[spec] = info
    np.testing.assert_allclose(out[1]["chi2"], out[0]["chi2"], rtol=1e-5)


def test_speculative_nonfinite_stamp_in_batch(ctx, gfo):
    # one stamp's data holds a NaN: that fit ends at its (clipped) start by the
    # damping cap; the other stamps of the batch fit as they do without it
    stamps = _stamps(85, 3)
    gb, lo, hi = _problem(ctx, gfo, stamps)
    start = to_dev(np.concatenate([s.start for s in stamps]), torch.float64)
    ref, rinfo = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, start, lo=lo, hi=hi, ftol=1e-6,
                            speculate=1)
    bad = gb.data.clone()
    bad[gb.batch.offsets["img"][1] + 5] = float("nan")
    th, info = ops.fit_lm(ctx, gb.batch, gb.psf, bad, gb.weight, start, lo=lo, hi=hi, ftol=1e-6, speculate=1)
    th, ref = th.cpu().numpy(), ref.cpu().numpy()
    po = gb.batch.offsets["par"]
    assert info["status"][1] == L.GF_ENOTCONV and info["reason"][1] == 4
    s1 = np.clip(np.concatenate([s.start for s in stamps]), lo.cpu().numpy(), hi.cpu().numpy())
    np.testing.assert_array_equal(th[po[1]:po[1] + 8], s1[po[1]:po[1] + 8])
    for s in (0, 2):
        np.testing.assert_array_equal(th[po[s]:po[s] + 8], ref[po[s]:po[s] + 8])
        assert info["chi2"][s] == rinfo["chi2"][s]


def test_start_pointer_matches_in_place(ctx, gfo):
    # gf_lm_opts.start: the start is read from its own buffer (left as it is)
    # and theta_io is output only; the fit is the in-place fit, bit for bit
    stamps = _stamps(86, 3)
    gb, lo, hi = _problem(ctx, gfo, stamps)
    st0 = np.concatenate([s.start for s in stamps])
    start = to_dev(st0, torch.float64)
    nb = len(stamps) * ops.LM_RESULT_DTYPE.itemsize
    ctx.bind_stream()
    for spec in (0, 1):
        print(f"start pointer, speculate={spec}", flush=True)
        o = L.gf_lm_opts_default()
        o.lo, o.hi, o.ftol, o.speculate = int(lo.data_ptr()), int(hi.data_ptr()), 1e-6, spec
        th_a = start.clone()
        res_a = torch.empty(nb, dtype=torch.uint8, device=ctx.device)
        L.gf_fit_lm(ctx.ptr, gb.batch.ptr, gb.psf.ptr, int(gb.data.data_ptr()), int(gb.weight.data_ptr()),
                    int(th_a.data_ptr()), o, int(res_a.data_ptr()))
        th_b = torch.full_like(start, float("nan"))
        res_b = torch.empty(nb, dtype=torch.uint8, device=ctx.device)
        o.start = int(start.data_ptr())
        L.gf_fit_lm(ctx.ptr, gb.batch.ptr, gb.psf.ptr, int(gb.data.data_ptr()), int(gb.weight.data_ptr()),
                    int(th_b.data_ptr()), o, int(res_b.data_ptr()))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(th_b.cpu().numpy(), th_a.cpu().numpy())
        ia, ib = ops.lm_info(res_a), ops.lm_info(res_b)
        for f in ("chi2", "iters", "nfev", "njev", "status", "reason"):
            np.testing.assert_array_equal(ib[f], ia[f], err_msg=f)
        np.testing.assert_array_equal(start.cpu().numpy(), st0)


def test_fit_lm_leaves_theta0_and_keeps_tail(ctx, gfo):
    # ops.fit_lm reads the start from theta0, which it leaves as it is; a
    # theta0 longer than the batch's parameters passes its tail through
    stamps = _stamps(87, 2)
    gb, lo, hi = _problem(ctx, gfo, stamps)
    st0 = np.concatenate([s.start for s in stamps])
    n = st0.size
    ext = np.concatenate([st0, [1.5, -2.5, 7.0]])
    t_ext = to_dev(ext, torch.float64)
    th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, t_ext, lo=lo, hi=hi, ftol=1e-6)
    ref, rinfo = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, t_ext[:n].clone(), lo=lo, hi=hi, ftol=1e-6)
    th = th.cpu().numpy()
    np.testing.assert_array_equal(t_ext.cpu().numpy(), ext)
    np.testing.assert_array_equal(th[n:], ext[n:])
    np.testing.assert_array_equal(th[:n], ref.cpu().numpy())
    np.testing.assert_array_equal(info["chi2"], rinfo["chi2"])
