"""The context's tuning table on a device: a context created with a tuning
file measures the FFT form of each one-workgroup side and the direct-path
PSF threshold on first use and writes the file; a second context reading it
takes the same choices and gives the same bits; every path agrees with the
oracle's convolution."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import _lib as L
from paper_1101_2254_amd import ops
from tests.gpu_common import GpuBatch, rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _stamps():
    g = synth.rng(9090)
    out = [synth.c3_stamp(g, N, i, 9090) for i, N in enumerate([32, 64, 96, 128, 128, 64])]
    # a 9 px PSF, where the direct-path threshold decides the path
    out[5].psf = synth.gaussian_psf(9, 1.3)
    return out


def _observed(gfo, stamps):
    data, weights = [], []
    for s, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64),
                      st.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, 40 + s)
        data.append(d)
        weights.append(w)
    return data, weights


def test_tuning_file_round_trip(tmp_path, gfo):
    path = str(tmp_path / "tune.json")
    stamps = _stamps()
    data, weights = _observed(gfo, stamps)
    lo = np.concatenate([synth.bounds(1, st.H, st.W)[0] for st in stamps])
    hi = np.concatenate([synth.bounds(1, st.H, st.W)[1] for st in stamps])
    start = np.concatenate([st.start for st in stamps])
    out = []
    for run in range(2):
        print(f"tuning context {run}", flush=True)
        ctx = ops.Context(0, autotune_cache=path)
        gb = GpuBatch(ctx, stamps, data=data, weights=weights)
        dk = L.gf_tune_direct_get(ctx.ptr)
        assert dk in range(1, 16, 2), dk
        sides = sorted({int(s) for u, s in zip(gb.psf.uses_fft, gb.psf.fft_side) if u})
        forms = {s: L.gf_tune_form_get(ctx.ptr, s) for s in sides}
        assert all(f in (1, 2) for f in forms.values()), forms
        assert os.path.exists(path)
        # each stamp on the path the table names: direct up to its PSF side
        # threshold, else the form of its FFT side
        for st, u, s in zip(stamps, gb.psf.uses_fft, gb.psf.fft_side):
            assert u == (0 if st.K <= dk else forms[int(s)])
        th, info = ops.fit_lm(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(start, torch.float64),
                              lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=1e-8)
        chi = ops.pairs_to_f64(ops.likelihood(ctx, gb.batch, gb.psf, gb.theta, gb.data, gb.weight, 5)).cpu().numpy()
        mins = {s: L.gf_tune_min_active_get(ctx.ptr, s) for s in sides}
        out.append((forms, mins, th.cpu().numpy(), info, chi, dk))
        torch.cuda.synchronize()
        ctx.close()
    tab = json.load(open(path))
    assert tab["arch"].startswith("gfx950")
    assert {int(k) for k in tab["form"]} >= set(out[0][0])
    # the second context read the table: same choices, same bits
    assert out[1][0] == out[0][0] and out[1][1] == out[0][1] and out[1][5] == out[0][5]
    assert tab["direct_max_k"] == out[0][5]   # measured on first use (the 9 px PSF)
    np.testing.assert_array_equal(out[1][2], out[0][2])
    np.testing.assert_array_equal(out[1][4], out[0][4])
    for k in ("chi2", "iters", "nfev"):
        np.testing.assert_array_equal(out[1][3][k], out[0][3][k])
    # the likelihood at the truth against the oracle (whichever form was chosen)
    gb_chi = out[0][4]
    for s, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64),
                      st.psf.astype(np.float32).astype(np.float64), 5)
        ref = gfo.chi2(data[s].astype(np.float32).astype(np.float64), weights[s].astype(np.float32).astype(np.float64), m)
        assert gb_chi[s] == pytest.approx(ref, rel=1e-5)


def test_autotune_call_and_errors(tmp_path):
    ctx = ops.Context(0, autotune_cache=str(tmp_path / "t.json"))
    L.gf_autotune(ctx.ptr, [48, 160])
    assert L.gf_tune_form_get(ctx.ptr, 48) in (1, 2) and L.gf_tune_form_get(ctx.ptr, 160) in (1, 2)
    assert L.gf_tune_form_get(ctx.ptr, 250) == 0          # not a one-workgroup side
    with pytest.raises(L.GfError) as e:
        L.gf_autotune(ctx.ptr, [250])
    assert e.value.status == L.GF_EINVAL
    with pytest.raises(L.GfError):
        L.gf_tune_form_set(ctx.ptr, 250, 2)
    # a context without a file measures nothing: untuned sides follow the
    # default rule
    c2 = ops.Context(0)
    assert L.gf_tune_form_get(c2.ptr, 48) == -1
    b = ops.Batch(c2, [34], [34], [15], [1])
    p = ops.Psf(c2, b, to_dev(np.full(225, 1 / 225.0, np.float32)), ops.GF_CONV_AUTO)
    assert list(p.uses_fft) == [2] and L.gf_tune_form_get(c2.ptr, 48) == -1
    # every side and the direct-path threshold
    L.gf_autotune(ctx.ptr, [])
    dk = L.gf_tune_direct_get(ctx.ptr)
    assert dk in range(1, 16, 2)
    assert json.load(open(str(tmp_path / "t.json")))["direct_max_k"] == dk
    L.gf_tune_direct_set(ctx.ptr, 9)
    assert L.gf_tune_direct_get(ctx.ptr) == 9
    with pytest.raises(L.GfError):
        L.gf_tune_direct_set(ctx.ptr, 8)
    b9 = ops.Batch(ctx, [40, 40], [40, 40], [9, 11], [1, 1])
    p9 = ops.Psf(ctx, b9, to_dev(np.full(81 + 121, 0.01, np.float32)), ops.GF_CONV_AUTO)
    assert list(p9.uses_fft)[0] == 0 and list(p9.uses_fft)[1] != 0
    assert L.gf_tune_direct_get(c2.ptr) == 7        # the default rule
    torch.cuda.synchronize()
    ctx.close()
    c2.close()
