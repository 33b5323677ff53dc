"""GPU parity of the spectral-line family against the FP64 reference
(oracle/line_ref.py): model spectra, chi^2 and whole LM fits on uneven
batches (ragged lengths, N below one chunk and below the LSF length, K = 1,
one to three lines)."""
import numpy as np
import pytest
import torch

import synth
from oracle import line_ref as LR
from paper_1101_2254_amd import ops
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("gpu lines: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _spectra(seed, shapes):
    """shapes: list of (N, n_lines, K or None)."""
    g = synth.rng(seed)
    out = []
    for i, (N, nl, K) in enumerate(shapes):
        sp = synth.line_spectrum(g, N, nl, i, seed)
        if K is not None:
            sp.lsf = synth.gaussian_lsf(K, 1.3) if K > 1 else np.ones(1)
        out.append(sp)
    return out


class LineSet:
    def __init__(self, ctx, spectra, noise=True, thetas=None):
        self.sp = spectra
        self.lb = ops.LineBatch(ctx, [s.N for s in spectra], [s.K for s in spectra], [s.nlines for s in spectra])
        self.lsf32 = [s.lsf.astype(np.float32) for s in spectra]
        self.lsf = to_dev(np.concatenate(self.lsf32))
        th = thetas if thetas is not None else [s.truth for s in spectra]
        self.th32 = [t.astype(np.float32) for t in th]
        self.theta = to_dev(np.concatenate(self.th32))
        self.d32, self.w32 = [], []
        for s, l32 in zip(spectra, self.lsf32):
            m = LR.model(s.truth.astype(np.float32).astype(np.float64), s.N, l32.astype(np.float64), 5)
            d, w = synth.add_noise_1d(m, s.noise_sigma, s.noise_seed) if noise else (m, np.ones(s.N))
            self.d32.append(d.astype(np.float32))
            self.w32.append(w.astype(np.float32))
        self.data = to_dev(np.concatenate(self.d32))
        self.weight = to_dev(np.concatenate(self.w32))

    def split(self, flat):
        o = self.lb.offsets["data"]
        f = flat.cpu().numpy() if isinstance(flat, torch.Tensor) else flat
        return [f[o[i]:o[i + 1]] for i in range(self.lb.n)]


SHAPES = [(1, 1, 1), (5, 1, 9), (37, 2, 15), (256, 1, 7), (300, 3, 21), (513, 2, 11), (1024, 3, 65),
          (2048, 1, 13), (777, 2, None), (64, 3, 3)]


@pytest.mark.parametrize("S", [1, 5])
def test_line_model_parity(ctx, S):
    ls = LineSet(ctx, _spectra(601, SHAPES), noise=False)
    print(f"line model S={S}", flush=True)
    out = ls.split(ops.line_model(ctx, ls.lb, ls.lsf, ls.theta, S))
    for i, s in enumerate(ls.sp):
        ref = LR.model(ls.th32[i].astype(np.float64), s.N, ls.lsf32[i].astype(np.float64), S)
        err = np.linalg.norm(out[i] - ref) / np.linalg.norm(ref)
        assert err <= 1e-5, (i, s.N, s.K, err)


def test_line_chi2_parity(ctx):
    ls = LineSet(ctx, _spectra(602, SHAPES))
    th = [t.copy() for t in ls.th32]
    for t in th:   # away from the truth as well
        t[1] += 0.3
    ls.theta = to_dev(np.concatenate(th))
    print("line chi2", flush=True)
    pairs = ops.line_chi2(ctx, ls.lb, ls.lsf, ls.theta, ls.data, ls.weight, 5)
    chi = ops.pairs_to_f64(pairs).cpu().numpy()
    for i, s in enumerate(ls.sp):
        m = LR.model(th[i].astype(np.float64), s.N, ls.lsf32[i].astype(np.float64), 5)
        ref = LR.chi2(ls.d32[i].astype(np.float64), ls.w32[i].astype(np.float64), m)
        # FP32 model error enters chi^2 through the cross term (Cauchy-Schwarz)
        wm = np.sqrt(np.sum(ls.w32[i] * m * m))
        assert abs(chi[i] - ref) <= 1e-5 * ref + 2 * 2e-6 * np.sqrt(ref) * wm + 1e-6, (i, chi[i], ref)
    assert torch.equal(pairs, ops.line_chi2(ctx, ls.lb, ls.lsf, ls.theta, ls.data, ls.weight, 5))


def _bounds(spectra):
    lo = np.concatenate([synth.line_bounds(s.nlines, s.N)[0] for s in spectra])
    hi = np.concatenate([synth.line_bounds(s.nlines, s.N)[1] for s in spectra])
    return lo, hi


def test_line_fit_parity(ctx):
    shapes = [(256, 1, None), (300, 2, None), (512, 3, None), (1024, 2, None), (2048, 1, None), (700, 3, None)]
    sp = _spectra(603, shapes)
    ls = LineSet(ctx, sp)
    lo, hi = _bounds(sp)
    start = np.concatenate([s.start for s in sp])
    opts = dict(ftol=1e-12, xtol=1e-10, max_iter=200)
    print("line fits", flush=True)
    th, info = ops.line_fit_lm(ctx, ls.lb, ls.lsf, ls.data, ls.weight, to_dev(start, torch.float64),
                               lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), **opts)
    th = th.cpu().numpy()
    po = ls.lb.offsets["par"]
    for i, s in enumerate(sp):
        l, h = synth.line_bounds(s.nlines, s.N)
        ref, rinfo = LR.fit_lm(s.start, ls.lsf32[i].astype(np.float64), ls.d32[i].astype(np.float64),
                               ls.w32[i].astype(np.float64), 5, lo=l, hi=h, **opts)
        got = th[po[i]:po[i + 1]]
        # at ftol 1e-12 the FP32 chi^2 cannot resolve the last decreases, so
        # the GPU may end by the damping cap once at the minimum (as the
        # image fits do); the oracle converges, and the two minima agree
        assert rinfo["status"] == 0, (i, rinfo)
        assert info["chi2"][i] == pytest.approx(rinfo["chi2"], rel=1e-5), i
        # parameters within 1e-4 relative (centres and widths on the scale of
        # the line width, amplitudes and continuum on the noise level)
        for k in range(s.nlines):
            a, mu, sg = ref[3 * k:3 * k + 3]
            assert abs(got[3 * k] - a) <= 1e-4 * max(abs(a), s.noise_sigma), (i, k)
            assert abs(got[3 * k + 1] - mu) <= 1e-4 * max(sg, 1.0), (i, k)
            assert abs(got[3 * k + 2] - sg) <= 1e-4 * max(sg, 1.0), (i, k)
        assert abs(got[-1] - ref[-1]) <= 1e-4 * max(abs(ref[-1]), s.noise_sigma), i
        assert np.all(got >= l) and np.all(got <= h)
    # at the throughput tolerance (ftol 1e-5) both converge, to the same chi^2
    th5, info5 = ops.line_fit_lm(ctx, ls.lb, ls.lsf, ls.data, ls.weight, to_dev(start, torch.float64),
                                 lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=1e-5)
    for i, s in enumerate(sp):
        l, h = synth.line_bounds(s.nlines, s.N)
        _, r5 = LR.fit_lm(s.start, ls.lsf32[i].astype(np.float64), ls.d32[i].astype(np.float64),
                          ls.w32[i].astype(np.float64), 5, lo=l, hi=h, ftol=1e-5)
        assert info5["status"][i] == 0 and r5["status"] == 0, (i, info5[i], r5)
        assert info5["chi2"][i] == pytest.approx(r5["chi2"], rel=1e-5), i
    # the same spectrum alone gives the same bits
    one = LineSet(ctx, [sp[2]])
    t1, i1 = ops.line_fit_lm(ctx, one.lb, one.lsf, one.data, one.weight, to_dev(sp[2].start, torch.float64),
                             lo=to_dev(synth.line_bounds(3, 512)[0], torch.float64),
                             hi=to_dev(synth.line_bounds(3, 512)[1], torch.float64), **opts)
    np.testing.assert_array_equal(t1.cpu().numpy(), th[po[2]:po[3]])
    assert i1["chi2"][0] == info["chi2"][2] and i1["iters"][0] == info["iters"][2]


def test_line_fit_edge_cases(ctx):
    # zero weights: chi^2 = 0 stops at once; truth start on noise-free data
    sp = _spectra(604, [(128, 2, None), (40, 1, 5)])
    ls = LineSet(ctx, sp, noise=False)
    w = torch.zeros_like(ls.weight)
    th, info = ops.line_fit_lm(ctx, ls.lb, ls.lsf, ls.data, w, to_dev(np.concatenate([s.start for s in sp]),
                                                                       torch.float64))
    assert np.all(info["status"] == 0) and np.all(info["reason"] == 3) and np.all(info["iters"] == 0)
    # noise-free data from the perturbed start: chi^2 falls to the FP32 floor
    # (where the relative-decrease test cannot fire, so the damping cap ends
    # the fit) and the parameters are back at the truth
    lo, hi = _bounds(sp)
    th, info = ops.line_fit_lm(ctx, ls.lb, ls.lsf, ls.data, ls.weight,
                               to_dev(np.concatenate([s.start for s in sp]), torch.float64),
                               lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64))
    assert np.all(info["chi2"] < 1e-6)
    truth = np.concatenate([s.truth for s in sp])
    np.testing.assert_allclose(th.cpu().numpy(), truth, rtol=2e-3, atol=2e-3)
    # free mask: amplitudes and continuum only, the rest stays
    free = np.concatenate([[1, 0, 0] * s.nlines + [1] for s in sp]).astype(np.uint8)
    st = np.concatenate([s.start for s in sp])
    th2, info2 = ops.line_fit_lm(ctx, ls.lb, ls.lsf, ls.data, ls.weight, to_dev(st, torch.float64),
                                 free=to_dev(free, torch.uint8), ftol=1e-12, xtol=1e-12)
    np.testing.assert_array_equal(th2.cpu().numpy()[free == 0], st[free == 0])


def test_line_fit_failed_factorisation(ctx):
    """A spectrum with one non-finite weight makes every damped Gram matrix
    non-finite, so each iteration's Cholesky fails and only raises the
    damping (the path where the whole workgroup re-reads the failure flag
    before the next solve).  The fit must end by the damping cap at the
    clipped start, like the oracle's, while the other spectra of the batch
    fit exactly as without it."""
    shapes = [(200, 2, None), (300, 1, None), (512, 3, None)]
    sp = _spectra(605, shapes)
    ls = LineSet(ctx, sp)
    lo, hi = _bounds(sp)
    start = np.concatenate([s.start for s in sp])
    opts = dict(ftol=1e-8, max_iter=100)
    ref_th, ref_info = ops.line_fit_lm(ctx, ls.lb, ls.lsf, ls.data, ls.weight, to_dev(start, torch.float64),
                                       lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), **opts)
    w = ls.weight.clone()
    w[ls.lb.offsets["data"][0] + 37] = float("nan")
    print("line fit with a non-finite weight", flush=True)
    th, info = ops.line_fit_lm(ctx, ls.lb, ls.lsf, ls.data, w, to_dev(start, torch.float64),
                               lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), **opts)
    po = ls.lb.offsets["par"]
    l0, h0 = synth.line_bounds(sp[0].nlines, sp[0].N)
    w0 = ls.w32[0].astype(np.float64).copy()
    w0[37] = np.nan
    r_th, r_info = LR.fit_lm(sp[0].start, ls.lsf32[0].astype(np.float64), ls.d32[0].astype(np.float64), w0, 5,
                             lo=l0, hi=h0, **opts)
    assert info["status"][0] == r_info["status"] == 6 and info["reason"][0] == r_info["reason"] == 4
    assert info["iters"][0] == r_info["iters"] == 14
    assert info["lambda"][0] == pytest.approx(r_info["lam"], rel=1e-12)
    # no trial point was formed: each iteration ended at the factorisation
    assert info["nfev"][0] == 1 and info["njev"][0] == 1
    np.testing.assert_array_equal(th.cpu().numpy()[po[0]:po[1]], r_th)
    # the other spectra are untouched by it
    np.testing.assert_array_equal(th.cpu().numpy()[po[1]:], ref_th.cpu().numpy()[po[1]:])
    for k in ("chi2", "iters", "nfev", "status"):
        np.testing.assert_array_equal(np.asarray(info[k])[1:], np.asarray(ref_info[k])[1:])
