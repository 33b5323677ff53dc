"""Multi-start fits on the GPU: grouped batches (several stamps sharing one
observation and PSF) fit exactly like the same stamps with the observation
copied per stamp; the start set and the per-group choice follow their
reference rules; the chosen fit is never worse than the single start."""
import numpy as np
import pytest
import torch

import synth
from oracle import gfo
from oracle import multistart_ref as MS
from paper_1101_2254_amd import ops
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

G, S = 6, 4


@pytest.fixture(scope="module")
def ctx():
    print("gpu multistart: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def galaxies():
    g = synth.rng(5150)
    sts = [synth.c3_stamp(g, int(g.choice([32, 48, 64])), i, 5150) for i in range(G)]
    data, weights = [], []
    for i, st in enumerate(sts):
        m = gfo.model(st.H, st.W, st.truth.astype(np.float32).astype(np.float64),
                      st.psf.astype(np.float32).astype(np.float64), 5)
        d, w = synth.add_gaussian_noise(m, 0.02, 700 + i)
        data.append(d.astype(np.float32))
        weights.append(w.astype(np.float32))
    return sts, data, weights


def test_multistart_grouped_fit(ctx, galaxies):
    sts, data, weights = galaxies
    print("expand starts", flush=True)
    theta0 = np.stack([st.start for st in sts])
    starts = ops.expand_starts(ctx, to_dev(theta0, torch.float64), S)
    np.testing.assert_array_equal(starts.cpu().numpy(), MS.expand_starts(theta0, S))

    H = [st.H for st in sts for _ in range(S)]
    K = [st.K for st in sts for _ in range(S)]
    group = [g for g in range(G) for _ in range(S)]
    lo = np.concatenate([synth.bounds(1, h, h)[0] for h in H])
    hi = np.concatenate([synth.bounds(1, h, h)[1] for h in H])
    opts = dict(lo=to_dev(lo, torch.float64), hi=to_dev(hi, torch.float64), ftol=1e-5)

    print("grouped fit", flush=True)
    gb = ops.Batch(ctx, H, H, K, [1] * (G * S), group=group)
    assert gb.n_groups == G and gb.sizes["n_img"] == sum(st.H * st.W for st in sts)
    taps = to_dev(np.concatenate([st.psf.astype(np.float32).ravel() for st in sts]))
    gpsf = ops.Psf(ctx, gb, taps)
    d = to_dev(np.concatenate([x.ravel() for x in data]))
    w = to_dev(np.concatenate([x.ravel() for x in weights]))
    th_g, res = ops.fit_lm(ctx, gb, gpsf, d, w, starts.reshape(-1).contiguous(), return_device=True, **opts)
    info_g = ops.lm_info(res)

    print("replicated fit", flush=True)
    pb = ops.Batch(ctx, H, H, K, [1] * (G * S))
    taps_r = to_dev(np.concatenate([sts[g].psf.astype(np.float32).ravel() for g in group]))
    ppsf = ops.Psf(ctx, pb, taps_r)
    d_r = to_dev(np.concatenate([data[g].ravel() for g in group]))
    w_r = to_dev(np.concatenate([weights[g].ravel() for g in group]))
    th_r, info_r = ops.fit_lm(ctx, pb, ppsf, d_r, w_r, starts.reshape(-1).contiguous(), **opts)
    assert torch.equal(th_g, th_r)
    for f in ("chi2", "iters", "nfev", "njev", "status"):
        np.testing.assert_array_equal(info_g[f], info_r[f], err_msg=f)

    print("group best", flush=True)
    best, idx = ops.group_best(ctx, gb, res, th_g)
    members = [list(range(g * S, g * S + S)) for g in range(G)]
    ref_idx = MS.group_best(members, info_g["chi2"], info_g["status"])
    np.testing.assert_array_equal(idx.cpu().numpy(), ref_idx)
    th = th_g.cpu().numpy().reshape(-1, 8)
    b = best.cpu().numpy()
    for g in range(G):
        np.testing.assert_array_equal(b[g, :8], th[ref_idx[g]])
        assert np.all(b[g, 8:] == 0)
        single = info_g["chi2"][g * S]
        if info_g["status"][g * S] == 0:
            assert info_g["chi2"][ref_idx[g]] <= single
