"""FP64 numpy reference of the learned proposal network (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests use it to check the GPU training and
inference kernels; the product never imports it.  It shares no code with the
GPU library.

Network (inputs 128 x 128, one channel, NHWC layout everywhere):
    4 x [3x3 convolution, stride 2, padding 1, ReLU]  channels 32, 32, 64, 64
        (128 -> 64 -> 32 -> 16 -> 8 pixels)
    flatten (y, x, c order) 4096 -> dense 256 -> ReLU -> dense 8
Loss: mean squared error over the batch and the 8 outputs.
Optimiser: Adam (Kingma & Ba 2015) with bias-corrected moments.

Parameters are a dict of float64 arrays: convolution weights w{i} of shape
[C_out, 3, 3, C_in] and biases b{i} [C_out] for i = 1..4, dense weights w5
[256, 4096], w6 [8, 256] and biases b5, b6.
"""
from __future__ import annotations

import numpy as np

CONV_CHANNELS = (1, 32, 32, 64, 64)
FC = (4096, 256, 8)
PARAM_ORDER = ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4", "w5", "b5", "w6", "b6")


def param_shapes(side: int = 128):
    """Shapes for inputs of side x side pixels (side divisible by 16)."""
    s = {}
    for i in range(4):
        cin, cout = CONV_CHANNELS[i], CONV_CHANNELS[i + 1]
        s[f"w{i + 1}"] = (cout, 3, 3, cin)
        s[f"b{i + 1}"] = (cout,)
    s["w5"] = (FC[1], (side // 16) ** 2 * CONV_CHANNELS[-1])
    s["b5"] = (FC[1],)
    s["w6"] = (FC[2], FC[1])
    s["b6"] = (FC[2],)
    return s


def init_params(seed: int = 0, side: int = 128):
    """He-uniform weights, zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for k, shp in param_shapes(side).items():
        if k.startswith("b"):
            p[k] = np.zeros(shp)
        else:
            fan_in = int(np.prod(shp[1:]))
            lim = np.sqrt(6.0 / fan_in)
            p[k] = g.uniform(-lim, lim, shp)
    return p


def conv_s2(x, w, b):
    """y[n, oy, ox, co] = b[co] + sum_{ky,kx,ci} w[co, ky, kx, ci] x[n, 2oy+ky-1, 2ox+kx-1, ci]
    (zero outside the input)."""
    n, h, wd, ci = x.shape
    co = w.shape[0]
    ho, wo = h // 2, wd // 2
    xp = np.zeros((n, h + 2, wd + 2, ci))
    xp[:, 1:h + 1, 1:wd + 1, :] = x
    y = np.zeros((n, ho, wo, co)) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * ho:2, kx:kx + 2 * wo:2, :]  # [n, ho, wo, ci]
            y += patch @ w[:, ky, kx, :].T
    return y


def conv_s2_backward(x, w, dy):
    """Gradients of conv_s2 with respect to x, w and b given dy."""
    n, h, wd, ci = x.shape
    ho, wo = h // 2, wd // 2
    xp = np.zeros((n, h + 2, wd + 2, ci))
    xp[:, 1:h + 1, 1:wd + 1, :] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * ho:2, kx:kx + 2 * wo:2, :]
            dw[:, ky, kx, :] = np.einsum("nyxo,nyxi->oi", dy, patch)
            dxp[:, ky:ky + 2 * ho:2, kx:kx + 2 * wo:2, :] += dy @ w[:, ky, kx, :]
    return dxp[:, 1:h + 1, 1:wd + 1, :], dw, dy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def forward(p, x):
    """x: [n, 128, 128, 1] -> (outputs [n, 8], cache)."""
    acts = [x]
    a = x
    for i in range(4):
        a = relu(conv_s2(a, p[f"w{i + 1}"], p[f"b{i + 1}"]))
        acts.append(a)
    f = a.reshape(a.shape[0], -1)
    h = relu(f @ p["w5"].T + p["b5"])  # w5 has as many columns as f (4096 for 128 x 128 inputs)
    y = h @ p["w6"].T + p["b6"]
    return y, (acts, f, h)


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(p, cache, y, t):
    """Gradients of mse(y, t) with respect to every parameter."""
    acts, f, h = cache
    n = y.shape[0]
    g = {}
    dy = 2.0 * (y - t) / y.size
    g["w6"] = dy.T @ h
    g["b6"] = dy.sum(0)
    dh = (dy @ p["w6"]) * (h > 0)
    g["w5"] = dh.T @ f
    g["b5"] = dh.sum(0)
    da = (dh @ p["w5"]).reshape(acts[4].shape)
    for i in range(4, 0, -1):
        dz = da * (acts[i] > 0)
        dx, g[f"w{i}"], g[f"b{i}"] = conv_s2_backward(acts[i - 1], p[f"w{i}"], dz)
        da = dx
    return g


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    pn, mn, vn = {}, {}, {}
    for k in p:
        mn[k] = b1 * m[k] + (1 - b1) * g[k]
        vn[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = mn[k] / (1 - b1 ** step)
        vh = vn[k] / (1 - b2 ** step)
        pn[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return pn, mn, vn


def normalise_input(stamps, border: int = 4):
    """asinh((x - sky) / sigma) with sky and sigma the mean and standard
    deviation of the outer `border`-pixel frame of each stamp."""
    n, h, w = stamps.shape
    mask = np.ones((h, w), bool)
    mask[border:h - border, border:w - border] = False
    fr = stamps[:, mask]
    sky = fr.mean(1)
    sig = fr.std(1)
    sig = np.where(sig > 0, sig, 1.0)
    return np.arcsinh((stamps - sky[:, None, None]) / sig[:, None, None])[..., None]


# ---------------------------------------------------------------- parameter coding
# Targets of a single Sersic component plus sky on a side-N stamp (theta =
# x0, y0, Ie, Re, n, q, phi, sky):
#   t0 = x0 - N/2, t1 = y0 - N/2,
#   t2, t3 = ln Ie, ln Re mapped linearly from [ln 0.5, ln 5] and [ln 2, ln N/4] onto [-1, 1],
#   t4 = n mapped from [0.5, 6] onto [-1, 1],
#   (t5, t6) = (1 - q)(cos 2 phi, sin 2 phi) / 0.8,
#   t7 = sky mapped from [0, 0.05] onto [-1, 1].
def _lin(v, a, b):
    return (2.0 * v - (a + b)) / (b - a)


def _unlin(t, a, b):
    return 0.5 * ((b - a) * t + (a + b))


def encode(theta, side):
    th = np.asarray(theta, np.float64).reshape(-1, 8)
    t = np.empty_like(th)
    t[:, 0] = th[:, 0] - side / 2
    t[:, 1] = th[:, 1] - side / 2
    t[:, 2] = _lin(np.log(th[:, 2]), np.log(0.5), np.log(5.0))
    t[:, 3] = _lin(np.log(th[:, 3]), np.log(2.0), np.log(side / 4))
    t[:, 4] = _lin(th[:, 4], 0.5, 6.0)
    t[:, 5] = (1 - th[:, 5]) * np.cos(2 * th[:, 6]) / 0.8
    t[:, 6] = (1 - th[:, 5]) * np.sin(2 * th[:, 6]) / 0.8
    t[:, 7] = _lin(th[:, 7], 0.0, 0.05)
    return t


def decode(t, side):
    """Inverse of encode; n clamped to [0.2, 10], 1 - q to [0, 0.95], phi in [0, pi)."""
    t = np.asarray(t, np.float64).reshape(-1, 8)
    th = np.empty_like(t)
    th[:, 0] = side / 2 + t[:, 0]
    th[:, 1] = side / 2 + t[:, 1]
    th[:, 2] = np.exp(_unlin(t[:, 2], np.log(0.5), np.log(5.0)))
    th[:, 3] = np.exp(_unlin(t[:, 3], np.log(2.0), np.log(side / 4)))
    th[:, 4] = np.clip(_unlin(t[:, 4], 0.5, 6.0), 0.2, 10.0)
    e = np.minimum(0.8 * np.hypot(t[:, 5], t[:, 6]), 0.95)
    th[:, 5] = 1 - e
    th[:, 6] = np.mod(0.5 * np.arctan2(t[:, 6], t[:, 5]), np.pi)
    th[:, 7] = _unlin(t[:, 7], 0.0, 0.05)
    return th


def draw_prior(key, counter, n, side):
    """Prior draws of the uneven-batch workload from Philox uniforms: stamp i
    uses blocks counter + 2i and + 2i + 1, uniforms u0..u7 in word order."""
    from .philox_ref import raw_blocks, uniform24
    u = uniform24(raw_blocks(key, counter, 2 * n)).reshape(n, 8)
    th = np.empty((n, 8))
    th[:, 0] = side / 2 + 2 * u[:, 5] - 1
    th[:, 1] = side / 2 + 2 * u[:, 6] - 1
    th[:, 2] = 0.5 * 10.0 ** u[:, 4]
    th[:, 3] = 2 + (side / 4 - 2) * u[:, 1]
    th[:, 4] = 0.5 + 5.5 * u[:, 0]
    th[:, 5] = 0.2 + 0.8 * u[:, 2]
    th[:, 6] = np.pi * u[:, 3]
    th[:, 7] = 0.05 * u[:, 7]
    return th
