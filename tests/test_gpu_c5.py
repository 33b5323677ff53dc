"""Learned starting points end to end on the GPU: stamps rendered on the
device line up with their parameters (checked against the FP64 oracle), a
short training run lowers the loss, and Levenberg-Marquardt started from the
network's proposals needs fewer iterations than from the image-moment
default guess while reaching the same final chi^2 (relative difference at
most 1e-5) on most stamps.

The comparison is statistical, on fresh stamps (seed 3000) that the network
never saw: the thresholds leave a wide margin below what a 32768-stamp,
three-epoch run reaches (iterations about 2.2x fewer, equal chi^2 on about
94% of stamps)."""
import numpy as np
import pytest
import torch

import synth
from oracle import cnn_ref as C
from oracle import gfo
from paper_1101_2254_amd import ops
from paper_1101_2254_amd import proposal as PR
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu

SIDE = 128


@pytest.fixture(scope="module")
def ctx():
    print("gpu c5: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def test_rendered_set_matches_oracle(ctx):
    print("rendered set vs oracle", flush=True)
    psfs = synth.psf_bank(6, 2000)
    rs = PR.RenderedSet(ctx, psfs, 9, SIDE, seed=2000)
    theta = rs.theta.cpu().numpy().astype(np.float64)
    ref_theta = C.draw_prior((2000, 0x9A1A), (0, 0, 0, 0), 9, SIDE)
    np.testing.assert_allclose(theta, ref_theta, rtol=2e-7, atol=1e-7)
    clean = rs.clean.cpu().numpy().reshape(9, SIDE, SIDE)
    for i in (0, 4, 8):                               # 8 uses PSF 8 mod 6 = 2
        m = gfo.model(SIDE, SIDE, theta[i], psfs[i % 6].astype(np.float32).astype(np.float64))
        assert rel_l2(clean[i], m) < 1e-5, i
    np.testing.assert_allclose(rs.targets.cpu().numpy(), C.encode(theta, SIDE), rtol=1e-6, atol=1e-6)
    # fresh noise per epoch, reproducible per (epoch, stamp) whatever the batch split
    a = rs.noisy(0, 9, epoch=0).cpu().numpy()
    b = np.concatenate([rs.noisy(0, 4, epoch=0).cpu().numpy(), rs.noisy(4, 5, epoch=0).cpu().numpy()])
    c = rs.noisy(0, 9, epoch=1).cpu().numpy()
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    sd = np.std(a - rs.clean.cpu().numpy())
    assert abs(sd - 0.02) < 0.001


@pytest.fixture(scope="module")
def trained(ctx):
    print("training the proposal network (32768 stamps, 3 epochs)", flush=True)
    rs = PR.RenderedSet(ctx, synth.psf_bank(2048, 2000), 32768, SIDE, seed=2000)
    net = PR.ProposalNet(ctx, SIDE, max_batch=256)
    net.init(2000)
    losses = PR.train(net, rs, epochs=3, batch=256, lr=2e-3)
    print(f"losses {losses}", flush=True)
    yield net, losses
    torch.cuda.synchronize()
    net.close()


def test_training_lowers_the_loss(trained):
    net, losses = trained
    assert net.steps == 3 * 128
    assert losses[-1] < 0.5 * losses[0]
    assert losses[-1] < 0.2


def test_cnn_seeded_lm_beats_default_guesses(ctx, trained):
    net, _ = trained
    n = 512
    print(f"evaluating on {n} fresh stamps", flush=True)
    ev = PR.RenderedSet(ctx, synth.psf_bank(n, 3000), n, SIDE, seed=3000)
    data = ev.noisy(0, n, epoch=0).clone()
    weight = torch.full_like(data, 1.0 / 0.02 ** 2)
    lo, hi = synth.bounds(1, SIDE, SIDE)
    lo_t = torch.from_numpy(np.tile(lo, n)).to(ctx.device)
    hi_t = torch.from_numpy(np.tile(hi, n)).to(ctx.device)
    start_d = PR.moments_guess(ctx, ev.batch, data)
    start_c = net.predict(data).reshape(-1).contiguous()
    _, info_d = ops.fit_lm(ctx, ev.batch, ev.psf, data, weight, start_d, lo=lo_t, hi=hi_t, ftol=1e-5)
    _, info_c = ops.fit_lm(ctx, ev.batch, ev.psf, data, weight, start_c, lo=lo_t, hi=hi_t, ftol=1e-5)
    it_d, it_c = info_d["iters"].mean(), info_c["iters"].mean()
    rel = (info_c["chi2"] - info_d["chi2"]) / info_d["chi2"]
    equal = np.mean(np.abs(rel) <= 1e-5)
    better_c, better_d = np.mean(rel < -1e-5), np.mean(rel > 1e-5)
    print(f"iterations default {it_d:.2f} cnn {it_c:.2f}; equal chi2 {equal:.3f}; "
          f"cnn lower {better_c:.3f}, default lower {better_d:.3f}", flush=True)
    assert it_c < 0.75 * it_d
    assert equal >= 0.85
    assert better_c >= better_d
    assert np.mean(info_c["status"] == 0) >= np.mean(info_d["status"] == 0) - 0.02
