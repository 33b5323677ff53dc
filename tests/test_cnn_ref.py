"""Pins of the FP64 reference of the proposal network (CPU)."""
import numpy as np
import pytest

from oracle import cnn_ref as C


def _conv_brute(x, w, b):
    n, h, wd, ci = x.shape
    co = w.shape[0]
    y = np.zeros((n, h // 2, wd // 2, co))
    for a in range(n):
        for oy in range(h // 2):
            for ox in range(wd // 2):
                for o in range(co):
                    acc = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            iy, ix = 2 * oy + ky - 1, 2 * ox + kx - 1
                            if 0 <= iy < h and 0 <= ix < wd:
                                acc += np.dot(w[o, ky, kx, :], x[a, iy, ix, :])
                    y[a, oy, ox, o] = acc
    return y


def test_conv_matches_brute_force():
    g = np.random.default_rng(1)
    x = g.standard_normal((2, 6, 8, 3))
    w = g.standard_normal((4, 3, 3, 3))
    b = g.standard_normal(4)
    np.testing.assert_allclose(C.conv_s2(x, w, b), _conv_brute(x, w, b), rtol=1e-12, atol=1e-12)


def test_conv_backward_is_the_adjoint():
    """<conv(x) - b, dy> = <x, dx> and = <w, dw> (bilinearity)."""
    g = np.random.default_rng(2)
    x = g.standard_normal((2, 8, 8, 3))
    w = g.standard_normal((5, 3, 3, 3))
    b = np.zeros(5)
    dy = g.standard_normal((2, 4, 4, 5))
    y = C.conv_s2(x, w, b)
    dx, dw, db = C.conv_s2_backward(x, w, dy)
    lhs = np.sum(y * dy)
    assert np.sum(x * dx) == pytest.approx(lhs, rel=1e-12)
    assert np.sum(w * dw) == pytest.approx(lhs, rel=1e-12)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2)))


def test_network_gradient_matches_central_differences():
    side = 16
    p = C.init_params(3, side)
    g = np.random.default_rng(4)
    x = g.standard_normal((3, side, side, 1))
    t = g.standard_normal((3, 8))
    y, cache = C.forward(p, x)
    grads = C.backward(p, cache, y, t)
    h = 1e-6
    for k in C.PARAM_ORDER:
        flat = p[k].reshape(-1)
        for idx in g.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = C.mse(C.forward(p, x)[0], t)
            flat[idx] = old - h
            lm = C.mse(C.forward(p, x)[0], t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[k].reshape(-1)[idx]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (k, idx)


def test_adam_first_step_closed_form():
    """With zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    p = {"a": np.array([1.0, -2.0, 3.0])}
    gr = {"a": np.array([0.5, -0.25, 0.0])}
    z = {"a": np.zeros(3)}
    pn, mn, vn = C.adam_step(p, gr, z, z, 1, 0.01)
    np.testing.assert_allclose(pn["a"], p["a"] - 0.01 * gr["a"] / (np.abs(gr["a"]) + 1e-8))
    np.testing.assert_allclose(mn["a"], 0.1 * gr["a"])
    np.testing.assert_allclose(vn["a"], 0.001 * gr["a"] ** 2)


def test_input_normalisation():
    st = np.zeros((1, 16, 16))
    st[0] += 2.0
    st[0, 0, :] = 4.0          # border values 2 and 4
    st[0, 8, 8] = 10.0
    z = C.normalise_input(st)
    mask = np.ones((16, 16), bool)
    mask[4:12, 4:12] = False
    fr = st[0][mask]
    assert z[0, 8, 8, 0] == pytest.approx(np.arcsinh((10 - fr.mean()) / fr.std()))
    assert z.shape == (1, 16, 16, 1)


def test_bf16_error_model_covers_rounded_network():
    """The element-wise error model used by the GPU forward test covers a CPU
    network that rounds every operand to BF16 (6 standard deviations), and
    it is tight enough to mean something (well below the outputs)."""
    from tests import cnn_bound as CB
    import synth
    side, n = 64, 16
    p = C.init_params(5, side)
    g = synth.rng(6)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.05 * g.standard_normal(p[k].shape)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    yy, xx = np.mgrid[0:side, 0:side]
    x = (0.02 * g.standard_normal((n, side, side))
         + np.exp(-((yy - 32.0) ** 2 / 50.0 + (xx - 30.0) ** 2 / 80.0))[None]).astype(np.float32)
    y, sd = CB.forward_error_sigma(p, x)
    ys = CB.forward_bf16(p, x)
    assert np.all(np.abs(ys - y) <= 6 * sd + 1e-6)
    assert sd.max() < 0.05 * np.abs(y).max()
    assert np.abs(ys - y).max() > 0.05 * sd.max()   # the rounding is really there
