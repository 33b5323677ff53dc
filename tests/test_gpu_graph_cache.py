"""The context keeps the captured LM iteration between gf_fit_lm calls and
replays it while the batch, PSF, caller pointers, workspace and options are
the same.  Every fit through a reused, recaptured or compacted graph must give
the bits a fresh context gives, including after the batch and PSF are
destroyed and replaced (possibly at the same host addresses)."""
import numpy as np
import pytest
import torch

import synth
from paper_1101_2254_amd import ops
from tests.gpu_common import GpuBatch, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("gpu graph cache: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _observed(gfo, stamps):
    data, weights = [], []
    for s in stamps:
        m = gfo.model(s.H, s.W, s.truth.astype(np.float32).astype(np.float64), s.psf.astype(np.float32).astype(np.float64),
                      5)
        d, w = synth.add_gaussian_noise(m, 0.02, s.noise_seed)
        data.append(d)
        weights.append(w)
    return data, weights


class Problem:
    def __init__(self, ctx, stamps, data, weights):
        self.gb = GpuBatch(ctx, stamps, data=data, weights=weights)
        lo = np.concatenate([synth.bounds(s.ncomp, s.H, s.W)[0] for s in stamps])
        hi = np.concatenate([synth.bounds(s.ncomp, s.H, s.W)[1] for s in stamps])
        self.lo, self.hi = to_dev(lo, torch.float64), to_dev(hi, torch.float64)
        self.start = to_dev(np.concatenate([s.start for s in stamps]), torch.float64)

    def fit(self, ctx, **kw):
        th, info = ops.fit_lm(ctx, self.gb.batch, self.gb.psf, self.gb.data, self.gb.weight, self.start, lo=self.lo,
                              hi=self.hi, **kw)
        return th.cpu().numpy(), info


def _same(a, b):
    np.testing.assert_array_equal(a[0], b[0])
    for f in ("chi2", "iters", "nfev", "njev", "status", "reason"):
        np.testing.assert_array_equal(a[1][f], b[1][f], err_msg=f)


def _fresh(stamps, data, weights, **kw):
    c = ops.Context(0)
    try:
        return Problem(c, stamps, data, weights).fit(c, **kw)
    finally:
        torch.cuda.synchronize()
        c.close()


def test_graph_reuse_matches_fresh_context(ctx, gfo):
    g = synth.rng(71)
    one = [synth.c1()]
    many = [synth.c3_stamp(g, int(N), i, 7100 + i) for i, N in enumerate([32, 48, 64, 32, 96, 48, 64, 32])]
    d1, w1 = _observed(gfo, one)
    d2, w2 = _observed(gfo, many)
    print("graph cache: reference fits in fresh contexts", flush=True)
    ref1 = _fresh(one, d1, w1, ftol=1e-5)
    ref2 = _fresh(many, d2, w2, ftol=1e-5)
    ref2b = _fresh(many, d2, w2, ftol=1e-8, poll_every=1)
    p1 = Problem(ctx, one, d1, w1)
    p2 = Problem(ctx, many, d2, w2)
    print("graph cache: repeated and alternating fits", flush=True)
    _same(p1.fit(ctx, ftol=1e-5), ref1)      # captured
    _same(p1.fit(ctx, ftol=1e-5), ref1)      # replayed
    _same(p2.fit(ctx, ftol=1e-5), ref2)      # another batch: recaptured
    _same(p2.fit(ctx, ftol=1e-5), ref2)
    # other options; with polling every iteration the batch is compacted
    # once half of its stamps are done (a graph of this call only)
    _same(p2.fit(ctx, ftol=1e-8, poll_every=1), ref2b)
    _same(p2.fit(ctx, ftol=1e-8, poll_every=1), ref2b)
    _same(p2.fit(ctx, ftol=1e-5), ref2)
    _same(p1.fit(ctx, ftol=1e-5), ref1)
    # a new start tensor is a new pointer
    p1.start = p1.start.clone()
    _same(p1.fit(ctx, ftol=1e-5), ref1)
    # another entry point grows (reallocates) the context's workspace
    g = synth.rng(72)
    big = [synth.c3_stamp(g, 256, i, 7200 + i) for i in range(48)]
    gbig = GpuBatch(ctx, big)
    ops.likelihood(ctx, gbig.batch, gbig.psf, gbig.theta, torch.zeros(gbig.batch.sizes["n_img"], device=ctx.device),
                   torch.ones(gbig.batch.sizes["n_img"], device=ctx.device), 5)
    _same(p1.fit(ctx, ftol=1e-5), ref1)
    # batch and PSF destroyed and replaced by another shape
    p1.gb.psf.close()
    p1.gb.batch.close()
    del p1
    p3 = Problem(ctx, many, d2, w2)
    _same(p3.fit(ctx, ftol=1e-5), ref2)
    _same(p3.fit(ctx, ftol=1e-5, use_graph=0), ref2)
    _same(p3.fit(ctx, ftol=1e-5), ref2)
