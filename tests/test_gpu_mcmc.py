"""GPU parity of the batched Metropolis sampler against the FP64 reference
chain (same Philox streams, chi^2 from the oracle).

Both sides take each accept decision from ln u < -(chi2' - chi2)/2 with
their own chi^2: the GPU's FP32 (compensated) chi^2 of a 64 x 64 stamp
agrees with the oracle's to about 1e-6 relative, i.e. ~5e-3 absolute at
chi^2 ~ 4e3.  A decision is therefore compared only where the reference's
margin |ln u + (chi2' - chi2)/2| exceeds 0.05; a chain whose decision falls
inside that band is followed no further (both outcomes are correct), and
at least 90 % of chain-steps must be compared."""
import numpy as np
import pytest
import torch

import synth
from oracle import gfo
from oracle import mcmc_ref as M
from paper_1101_2254_amd import ops
from tests.gpu_common import GpuBatch, to_dev

pytestmark = pytest.mark.gpu

N, K, CHAINS, STEPS = 64, 15, 16, 12
KEY, STREAM = (4004, 17), 5


@pytest.fixture(scope="module")
def ctx():
    print("gpu mcmc: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def setup(ctx):
    truth = np.array([32.3, 31.7, 1.0, 6.0, 2.5, 0.7, np.pi / 6, 0.01])
    psf = synth.moffat_psf(K, 3.0, 3.0)
    m = gfo.model(N, N, truth, psf.astype(np.float32).astype(np.float64), 5)
    d, w = synth.add_gaussian_noise(m, 0.02, 77)
    d32, w32 = d.astype(np.float32), w.astype(np.float32)
    g = synth.rng(99)
    th0 = np.tile(truth, (CHAINS, 1)) * (1 + 0.01 * g.standard_normal((CHAINS, 8)))
    scale = np.tile(np.abs(truth) * 0.004 + 1e-4, (CHAINS, 1))
    stamp = synth.Stamp(N, N, psf, truth, truth, 0.02)
    gb = GpuBatch(ctx, [stamp] * CHAINS, data=[d32], weights=[w32], shared=True)
    return gb, d32, w32, psf, th0, scale


def test_mcmc_matches_reference_chain(ctx, setup):
    gb, d32, w32, psf, th0, scale = setup
    lo, hi = synth.bounds(1, N, N)
    print("gpu chains", flush=True)
    th, c2, samples, acc = ops.mcmc_run(ctx, gb.batch, gb.psf, gb.data, gb.weight, to_dev(th0.ravel(), torch.float64),
                                        to_dev(scale.ravel(), torch.float64), STEPS, key=KEY, stream=STREAM,
                                        lo=to_dev(np.tile(lo, CHAINS), torch.float64),
                                        hi=to_dev(np.tile(hi, CHAINS), torch.float64))
    samples = samples.cpu().numpy().reshape(STEPS, CHAINS, 8)
    p64 = psf.astype(np.float32).astype(np.float64)
    d64, w64 = d32.astype(np.float64), w32.astype(np.float64)

    def chi2_fn(c, t):
        return gfo.chi2(d64, w64, gfo.model(N, N, t, p64, 5))

    print("reference chains", flush=True)
    st, ch, ok, margin = M.run(th0, scale, STEPS, chi2_fn, KEY, stream=STREAM, lo=np.tile(lo, (CHAINS, 1)),
                               hi=np.tile(hi, (CHAINS, 1)))
    compared = 0
    for c in range(CHAINS):
        for t in range(STEPS):
            if margin[t, c] < 0.05:
                break
            np.testing.assert_allclose(samples[t, c], st[t, c].astype(np.float32), rtol=2e-7, atol=1e-6,
                                       err_msg=f"chain {c} step {t}")
            compared += 1
        else:
            np.testing.assert_allclose(th.cpu().numpy()[8 * c:8 * c + 8], st[-1, c], rtol=1e-12, atol=0)
            assert c2.cpu().numpy()[c] == pytest.approx(ch[-1, c], rel=1e-5)
    assert compared >= 0.9 * CHAINS * STEPS, compared
    assert 0 < ok.mean() < 1


def test_mcmc_continuation_and_thinning(ctx, setup):
    """Steps 0..5 then 6..11 (step0 = 6) give the same chain as 12 at once;
    thin = 3 keeps every third state; the graph and plain launches agree."""
    gb, d32, w32, psf, th0, scale = setup
    t0, s0 = to_dev(th0.ravel(), torch.float64), to_dev(scale.ravel(), torch.float64)
    a_th, a_c2, a_s, a_acc = ops.mcmc_run(ctx, gb.batch, gb.psf, gb.data, gb.weight, t0, s0, 12, key=KEY, stream=2)
    b_th, _, b_s1, b_acc1 = ops.mcmc_run(ctx, gb.batch, gb.psf, gb.data, gb.weight, t0, s0, 6, key=KEY, stream=2)
    c_th, c_c2, b_s2, b_acc2 = ops.mcmc_run(ctx, gb.batch, gb.psf, gb.data, gb.weight, b_th, s0, 6, key=KEY,
                                            stream=2, step0=6)
    assert torch.equal(a_th, c_th) and torch.equal(a_c2, c_c2)
    assert torch.equal(a_s, torch.cat([b_s1, b_s2]))
    assert torch.equal(a_acc, b_acc1 + b_acc2)
    _, _, t_s, _ = ops.mcmc_run(ctx, gb.batch, gb.psf, gb.data, gb.weight, t0, s0, 12, key=KEY, stream=2, thin=3)
    assert torch.equal(t_s, a_s[2::3])
    p_th, _, p_s, _ = ops.mcmc_run(ctx, gb.batch, gb.psf, gb.data, gb.weight, t0, s0, 12, key=KEY, stream=2,
                                   use_graph=False)
    assert torch.equal(p_th, a_th) and torch.equal(p_s, a_s)
