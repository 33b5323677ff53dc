"""gf_chi2_noalloc (the step-3 entry point that allocates nothing) through
the C ABI against gf_chi2: the same bits, on two calls in a row with the
second batch smaller than the first, and a batch above the fixed array's
size refused before anything runs."""
import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import _lib as L
from paper_1101_2254_amd import ops
from tests.gpu_common import GpuBatch, to_dev

pytestmark = pytest.mark.gpu


def _case(ctx, gfo, sizes, seed):
    g = synth.rng(seed)
    stamps = [synth.c3_stamp(g, N, i, seed) for i, N in enumerate(sizes)]
    data, weights = [], []
    for s, st in enumerate(stamps):
        m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64),
                      st.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, seed + s)
        w[: st.H // 4, :] = 0.0                      # masked rows
        data.append(d)
        weights.append(w)
    gb = GpuBatch(ctx, stamps, thetas=[st.start for st in stamps], data=data, weights=weights)
    mp = ops.eval_model(ctx, gb.batch, gb.theta, 5)
    mc = ops.convolve_psf(ctx, gb.batch, gb.psf, mp)
    return gb, mc


def test_chi2_noalloc_matches_chi2(gfo):
    ctx = ops.Context(0)
    # two calls in a row through the C ABI: the second batch is smaller, so
    # the array still holds the first call's partials beyond its own
    for sizes, seed in (([256, 192, 128, 96, 64, 32, 256, 48], 71), ([64, 32], 72)):
        gb, mc = _case(ctx, gfo, sizes, seed)
        print(f"noalloc chi2 on {len(sizes)} stamps", flush=True)
        ref, r_ref = ops.chi2(ctx, gb.batch, mc, gb.theta, gb.data, gb.weight, want_resid=True)
        pairs = torch.full((gb.n, 2), float("nan"), dtype=torch.float32, device=ctx.device)
        resid = torch.full_like(r_ref, float("nan"))
        ctx.bind_stream()
        L.gf_chi2_noalloc(ctx.ptr, gb.batch.ptr, int(mc.data_ptr()), int(gb.theta.data_ptr()),
                          int(gb.data.data_ptr()), int(gb.weight.data_ptr()), int(resid.data_ptr()),
                          int(pairs.data_ptr()))
        torch.cuda.synchronize()
        assert torch.equal(pairs, ref)
        assert torch.equal(resid, r_ref)
        # the tensor-level binding, without the residual
        p2, none = ops.chi2_noalloc(ctx, gb.batch, mc, gb.theta, gb.data, gb.weight)
        assert none is None and torch.equal(p2, ref)
        # and the result is the oracle's chi^2 of the same FP32 model
        chi = ops.pairs_to_f64(pairs).cpu().numpy()
        ms = gb.split_pix(mc)
        for s, st in enumerate(gb.stamps):
            mm = ms[s].astype(np.float64) + np.float64(gb.th32[s][-1])
            assert chi[s] == pytest.approx(gfo.chi2(gb.d32[s], gb.w32[s], mm), rel=1e-6)
    torch.cuda.synchronize()
    ctx.close()


def test_chi2_noalloc_refuses_a_batch_above_its_array():
    ctx = ops.Context(0)
    # 129 stamps of 2048 x 2048: 132096 chunks of 4096 pixels > 131072
    b = ops.Batch(ctx, [2048] * 129, [2048] * 129, [1] * 129, [1] * 129)
    dummy = torch.zeros(16, dtype=torch.float32, device=ctx.device)
    p = int(dummy.data_ptr())
    with pytest.raises(L.GfError) as e:
        L.gf_chi2_noalloc(ctx.ptr, b.ptr, p, p, p, p, 0, p)
    assert e.value.status == L.GF_ESHAPE
    assert "131072" in L.lib().gf_last_error(ctx.ptr).decode()
    torch.cuda.synchronize()
    b.close()
    ctx.close()
