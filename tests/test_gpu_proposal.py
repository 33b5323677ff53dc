"""GPU parity of the starting-point path: Philox4x64-10 raw blocks against
numpy (bit-exact), Gaussian noise and prior draws against the FP64
references, the parameter coding, the image-moment guess against its FP64
reference, and the proposal network's forward pass, gradients and Adam
steps against the numpy FP64 network.

Network tolerances: the GPU rounds operands and activations to BF16 (unit
roundoff 2^-9) and accumulates in FP32.  Rounding errors of independent
operands do not grow with the dot-product length in the relative L2 sense;
each layer adds about 2^-9 * sqrt(2) ~ 3e-3, so six layers and the input
coding give about 1e-2.  The tests hold the outputs to 3e-2 and each
gradient tensor to 5e-2 relative L2.  The Adam update is FP32 element-wise
arithmetic on the same gradients (1e-5 relative).
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cnn_ref as C
from oracle import gfo
from oracle import moments_ref as MR
from oracle import philox_ref as PX
from paper_1101_2254_amd import ops
from paper_1101_2254_amd import proposal as PR
from tests.gpu_common import rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("gpu proposal: creating context on cuda:0", flush=True)
    c = ops.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("key,ctr,nb", [((0x1234, 0xABCDEF), (5, 0, 0, 0), 1000),
                                        ((2000, 1), ((1 << 64) - 300, 7, 0, 3), 1000)])
def test_philox_blocks_match_numpy(ctx, key, ctr, nb):
    print(f"philox key={key} ctr={ctr}", flush=True)
    got = _u64(PR.philox(ctx, key, ctr, nb)).reshape(-1)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                         counter=np.array(PX.counter_add(ctr, -1), dtype=np.uint64))
    assert np.array_equal(got, g.random_raw(4 * nb))


@pytest.mark.parametrize("n", [1, 4, 4003])
def test_normal_noise(ctx, n):
    print(f"normal noise n={n}", flush=True)
    key, ctr = (3000, 5), (17, 0, 0, 0)
    clean = np.linspace(-1, 1, n).astype(np.float32)
    got = PR.normal_noise(ctx, n, 0.25, key, ctr, clean=to_dev(clean))[:n].cpu().numpy()
    ref = clean.astype(np.float64) + 0.25 * PX.normals(key, ctr, n)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-7)


def test_prior_draw_and_coding(ctx):
    print("prior draw and coding", flush=True)
    n, side, key, ctr = 300, 128, (2000, 0x9A1A), (64, 0, 0, 0)
    th = PR.draw_prior(ctx, n, side, key, ctr)
    ref = C.draw_prior(key, ctr, n, side)
    np.testing.assert_allclose(th.cpu().numpy(), ref, rtol=2e-7, atol=1e-7)
    t = PR.encode(ctx, th.reshape(-1), side)
    tref = C.encode(th.cpu().numpy().astype(np.float64), side)
    np.testing.assert_allclose(t.cpu().numpy(), tref, rtol=1e-6, atol=1e-6)
    back = PR.decode(ctx, t, side).cpu().numpy()
    bref = C.decode(t.cpu().numpy().astype(np.float64), side)
    np.testing.assert_allclose(back, bref, rtol=1e-12, atol=1e-12)


def _moment_stamps():
    g = synth.rng(77)
    out = []
    for i, N in enumerate([32, 48, 64, 96, 128, 192, 256, 128, 64, 32]):
        st = synth.c3_stamp(g, N, i, 77)
        m = gfo.model(N, N, st.truth, st.psf)
        d = synth.add_gaussian_noise(m, 0.02, 9000 + i)[0].astype(np.float32)
        out.append((st, d))
    return out


def test_moments_guess_matches_reference(ctx):
    print("moments guess", flush=True)
    items = _moment_stamps()
    sts = [s for s, _ in items]
    b = ops.Batch(ctx, [s.H for s in sts], [s.W for s in sts], [s.K for s in sts], [1] * len(sts))
    data = to_dev(np.concatenate([d.ravel() for _, d in items]))
    th = PR.moments_guess(ctx, b, data).cpu().numpy().reshape(-1, 8)
    for i, (st, d) in enumerate(items):
        ref = MR.guess(d.astype(np.float64))
        for p in (0, 1, 2, 3, 4, 5, 7):
            assert th[i, p] == pytest.approx(ref[p], rel=1e-6, abs=1e-9), (i, p, th[i], ref)
        if ref[5] < 0.95:
            dphi = abs((th[i, 6] - ref[6] + math.pi / 2) % math.pi - math.pi / 2)
            assert dphi < 1e-6, (i, th[i, 6], ref[6])


def _net_inputs(n, side, seed):
    """Stamps of a few Gaussian blobs on a noisy sky."""
    g = synth.rng(seed)
    yy, xx = np.mgrid[0:side, 0:side].astype(float)
    x = np.empty((n, side, side))
    for i in range(n):
        img = g.uniform(0, 0.05) + 0.02 * g.standard_normal((side, side))
        for _ in range(3):
            cx, cy, s, a = g.uniform(side * 0.3, side * 0.7, 2).tolist() + [g.uniform(2, side / 6), g.uniform(0.2, 3)]
            img += a * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * s * s))
        x[i] = img
    return x.astype(np.float32)


def _flat(p):
    return np.concatenate([p[k].reshape(-1) for k in C.PARAM_ORDER])


def _unflat(v, side):
    out, o = {}, 0
    for k, shp in C.param_shapes(side).items():
        n = int(np.prod(shp))
        out[k] = v[o:o + n].reshape(shp)
        o += n
    return out


@pytest.fixture(scope="module")
def net_case(ctx):
    side, n = 128, 12
    p = C.init_params(11, side)
    g = synth.rng(12)
    for k in p:                                  # non-zero biases exercise the epilogue
        if k.startswith("b"):
            p[k] = 0.05 * g.standard_normal(p[k].shape)
    p32 = {k: v.astype(np.float32) for k, v in p.items()}
    x = _net_inputs(n, side, 13)
    t = g.uniform(-1, 1, (n, 8)).astype(np.float32)
    net = PR.ProposalNet(ctx, side, max_batch=16)
    net.set_params(to_dev(_flat(p32)))
    yield side, n, p32, x, t, net
    torch.cuda.synchronize()
    net.close()


def test_network_parameter_round_trip(net_case):
    side, n, p32, x, t, net = net_case
    assert net.n_params == sum(int(np.prod(s)) for s in C.param_shapes(side).values())
    assert np.array_equal(net.get_params().cpu().numpy(), _flat(p32))


def test_network_forward(net_case):
    print("network forward", flush=True)
    side, n, p32, x, t, net = net_case
    got = net.forward(to_dev(x)).cpu().numpy()
    p64 = {k: v.astype(np.float64) for k, v in p32.items()}
    ref, _ = C.forward(p64, C.normalise_input(x.astype(np.float64)))
    assert rel_l2(got, ref) < 3e-2, rel_l2(got, ref)


def test_network_forward_elementwise(net_case):
    """Every output of the forward pass within 6 standard deviations of the
    BF16 rounding model (tests/cnn_bound.py, itself checked on the CPU
    against a network that rounds every operand) of the FP64 reference."""
    from tests import cnn_bound as CB
    side, n, p32, x, t, net = net_case
    got = net.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    p64 = {k: v.astype(np.float64) for k, v in p32.items()}
    ref, sd = CB.forward_error_sigma(p64, x)
    err = np.abs(got - ref)
    print("forward: max |err| / sd", float((err / sd).max()), "max sd", float(sd.max()), flush=True)
    assert np.all(err <= 6.0 * sd + 1e-6), (err / sd).max()


def test_network_gradients(net_case):
    print("network gradients", flush=True)
    side, n, p32, x, t, net = net_case
    g, loss = net.gradients(to_dev(x), to_dev(t))
    p64 = {k: v.astype(np.float64) for k, v in p32.items()}
    y, cache = C.forward(p64, C.normalise_input(x.astype(np.float64)))
    gref = C.backward(p64, cache, y, t.astype(np.float64))
    assert float(loss.item()) == pytest.approx(C.mse(y, t), rel=3e-2)
    gg = _unflat(g.cpu().numpy(), side)
    for k in C.PARAM_ORDER:
        assert rel_l2(gg[k], gref[k]) < 5e-2, (k, rel_l2(gg[k], gref[k]))


def test_adam_steps(ctx, net_case):
    print("adam steps", flush=True)
    side, n, p32, x, t, net = net_case
    net.set_params(to_dev(_flat(p32)))
    xd, td = to_dev(x), to_dev(t)
    p = {k: v.astype(np.float64) for k, v in p32.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    lr = 1e-3
    for step in (1, 2):
        g, _ = net.gradients(xd, td)                 # the gradients the step will use (deterministic)
        gd = _unflat(g.cpu().numpy().astype(np.float64), side)
        net.train_step(xd, td, lr)
        p, m, v = C.adam_step(p, gd, m, v, step, lr)
        got = _unflat(net.get_params().cpu().numpy(), side)
        for k in C.PARAM_ORDER:
            np.testing.assert_allclose(got[k], p[k], rtol=1e-5, atol=1e-7, err_msg=f"{k} step {step}")
        p = {k: got[k].astype(np.float64) for k in p}   # continue from the FP32 state
    assert net.steps == 2
    net.set_params(to_dev(_flat(p32)))


def test_network_batches_are_independent(net_case):
    """The forward pass of a stamp does not depend on its batch neighbours or
    on how a long input is split into max_batch chunks."""
    side, n, p32, x, t, net = net_case
    xx = np.concatenate([x, x[::-1], x[:5]])      # 29 stamps: chunks of 16 + 13
    y = net.forward(to_dev(xx)).cpu().numpy()
    assert np.array_equal(y[:n], y[n:2 * n][::-1])
    assert np.array_equal(y[:5], y[2 * n:])
