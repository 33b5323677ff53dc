"""Starting points for single-Sersic fits: the image-moment default guess and
a learned proposal network trained on stamps rendered on the device.

The paper's outlook (Sec. 5) points out that a local optimiser only finds the
minimum near its start and that better strategies avoid local minima and
unphysical results; a good start also cuts the number of LM iterations,
which is where the device time of a batch goes.  Everything here marshals
tensors into ``libgf`` calls (moments, network, Philox noise, prior draws,
rendering through the step 1-2 kernels); no step runs in torch.

Parameter vector per stamp: ``[x0, y0, Ie, Re, n, q, phi, sky]``.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib as L
from .ops import Batch, Context, Psf, _need, _ptr, model as render_model

OUT = 8


def moments_guess(ctx: Context, batch: Batch, data: torch.Tensor) -> torch.Tensor:
    """Default starting points (gf_moments_guess) as a float64 tensor [n_par]."""
    _need(data, torch.float32, batch.sizes["n_img"], "data")
    theta = torch.empty(batch.sizes["n_par"], dtype=torch.float64, device=ctx.device)
    ctx.bind_stream()
    L.gf_moments_guess(ctx.ptr, batch.ptr, _ptr(data), _ptr(theta))
    return theta


def philox(ctx: Context, key, counter, n_blocks: int) -> torch.Tensor:
    """Raw Philox4x64-10 blocks as int64 tensor [n_blocks, 4] (bit pattern of the uint64 words)."""
    out = torch.empty((max(n_blocks, 1), 4), dtype=torch.int64, device=ctx.device)
    ctx.bind_stream()
    L.gf_philox(ctx.ptr, int(key[0]), int(key[1]), counter, int(n_blocks), _ptr(out))
    return out[:n_blocks]


def normal_noise(ctx: Context, n: int, sigma: float, key, counter, clean=None, out=None) -> torch.Tensor:
    if clean is not None:
        _need(clean, torch.float32, n, "clean")
    out = torch.empty(max(n, 1), dtype=torch.float32, device=ctx.device) if out is None else _need(
        out, torch.float32, n, "out")
    ctx.bind_stream()
    L.gf_normal_noise(ctx.ptr, int(n), float(sigma), int(key[0]), int(key[1]), counter, _ptr(clean), _ptr(out))
    return out


def draw_prior(ctx: Context, n: int, side: int, key, counter=(0, 0, 0, 0), out=None) -> torch.Tensor:
    """Single-Sersic parameters [n, 8] (float32) drawn on the device from the uneven-batch prior box."""
    out = torch.empty((max(n, 1), OUT), dtype=torch.float32, device=ctx.device) if out is None else out
    ctx.bind_stream()
    L.gf_draw_prior(ctx.ptr, int(n), int(side), int(key[0]), int(key[1]), counter, _ptr(out))
    return out[:n]


def encode(ctx: Context, theta: torch.Tensor, side: int, out=None) -> torch.Tensor:
    n = theta.numel() // OUT
    _need(theta, torch.float32, n * OUT, "theta")
    out = torch.empty((max(n, 1), OUT), dtype=torch.float32, device=ctx.device) if out is None else out
    ctx.bind_stream()
    L.gf_cnn_encode(ctx.ptr, n, int(side), _ptr(theta), _ptr(out))
    return out[:n]


def decode(ctx: Context, targets: torch.Tensor, side: int) -> torch.Tensor:
    n = targets.numel() // OUT
    _need(targets, torch.float32, n * OUT, "targets")
    theta = torch.empty((max(n, 1), OUT), dtype=torch.float64, device=ctx.device)
    ctx.bind_stream()
    L.gf_cnn_decode(ctx.ptr, n, int(side), _ptr(targets), _ptr(theta))
    return theta[:n]


class ProposalNet:
    """The proposal network (gf_cnn): BF16 matrix-core forward/backward, Adam."""

    def __init__(self, ctx: Context, side: int = 128, max_batch: int = 256):
        self.ctx, self.side, self.max_batch = ctx, int(side), int(max_batch)
        ctx.bind_stream()
        self.ptr = L.gf_cnn_create(ctx.ptr, self.side, self.max_batch)
        self.n_params = L.gf_cnn_param_count(self.ptr)
        self._loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)

    def init(self, key: int):
        self.ctx.bind_stream()
        L.gf_cnn_init(self.ctx.ptr, self.ptr, int(key))

    def set_params(self, params: torch.Tensor):
        _need(params, torch.float32, self.n_params, "params")
        self.ctx.bind_stream()
        L.gf_cnn_set_params(self.ctx.ptr, self.ptr, _ptr(params))

    def get_params(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.ctx.device)
        self.ctx.bind_stream()
        L.gf_cnn_get_params(self.ctx.ptr, self.ptr, _ptr(out))
        return out

    def _stamps(self, stamps):
        n = stamps.numel() // (self.side * self.side)
        _need(stamps, torch.float32, n * self.side * self.side, "stamps")
        return n

    def forward(self, stamps: torch.Tensor) -> torch.Tensor:
        n = self._stamps(stamps)
        out = torch.empty((max(n, 1), OUT), dtype=torch.float32, device=self.ctx.device)
        self.ctx.bind_stream()
        L.gf_cnn_forward(self.ctx.ptr, self.ptr, _ptr(stamps), n, _ptr(out))
        return out[:n]

    def gradients(self, stamps: torch.Tensor, targets: torch.Tensor):
        n = self._stamps(stamps)
        _need(targets, torch.float32, n * OUT, "targets")
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.ctx.device)
        self.ctx.bind_stream()
        L.gf_cnn_gradients(self.ctx.ptr, self.ptr, _ptr(stamps), _ptr(targets), n, _ptr(g), _ptr(self._loss))
        return g, self._loss.clone()

    def train_step(self, stamps: torch.Tensor, targets: torch.Tensor, lr: float) -> torch.Tensor:
        """One Adam step; returns the batch loss as a device tensor (no host sync)."""
        n = self._stamps(stamps)
        _need(targets, torch.float32, n * OUT, "targets")
        self.ctx.bind_stream()
        L.gf_cnn_train_step(self.ctx.ptr, self.ptr, _ptr(stamps), _ptr(targets), n, float(lr), _ptr(self._loss))
        return self._loss

    @property
    def steps(self) -> int:
        return L.gf_cnn_steps(self.ptr)

    def predict(self, stamps: torch.Tensor) -> torch.Tensor:
        """Starting points [n, 8] float64 decoded from the network outputs."""
        return decode(self.ctx, self.forward(stamps), self.side)

    def close(self):
        if getattr(self, "ptr", None):
            L.gf_cnn_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RenderedSet:
    """n noise-free side x side single-Sersic stamps rendered on the device
    (prior draw -> Sersic evaluation on the padded grid -> PSF convolution ->
    sky), kept resident in HBM with their coded targets.  Stamp i uses PSF
    i mod len(psfs); noise is added per batch by :meth:`noisy` from Philox
    keyed on (seed, epoch), so each epoch sees fresh noise."""

    def __init__(self, ctx: Context, psfs, n: int, side: int = 128, seed: int = 2000, sigma: float = 0.02,
                 oversample: int = 5):
        self.ctx, self.n, self.side, self.seed, self.sigma = ctx, int(n), int(side), int(seed), float(sigma)
        nb = len(psfs)
        self.batch = Batch(ctx, [side] * nb, [side] * nb, [p.shape[0] for p in psfs], [1] * nb)
        taps = np.concatenate([np.asarray(p, np.float32).reshape(-1) for p in psfs])
        self.psf = Psf(ctx, self.batch, torch.from_numpy(taps).to(ctx.device))
        px = side * side
        dev = ctx.device
        self.clean = torch.empty(self.n * px, dtype=torch.float32, device=dev)
        self.theta = torch.empty((self.n, OUT), dtype=torch.float32, device=dev)
        self.targets = torch.empty((self.n, OUT), dtype=torch.float32, device=dev)
        self.psf_index = np.arange(self.n) % nb
        th = torch.empty((nb, OUT), dtype=torch.float32, device=dev)
        for c0 in range(0, self.n, nb):
            m = min(nb, self.n - c0)
            draw_prior(ctx, nb, side, (self.seed, 0x9a1a), (2 * c0, 0, 0, 0), out=th)
            out = render_model(ctx, self.batch, self.psf, th.reshape(-1), oversample)
            self.clean[c0 * px:(c0 + m) * px].copy_(out[:m * px])
            self.theta[c0:c0 + m].copy_(th[:m])
        encode(ctx, self.theta.reshape(-1), side, out=self.targets)

    def noisy(self, start: int, count: int, epoch: int, out=None) -> torch.Tensor:
        px = self.side * self.side
        return normal_noise(self.ctx, count * px, self.sigma, (self.seed, epoch + 1), (start * px // 4, 0, 0, 0),
                            clean=self.clean[start * px:(start + count) * px], out=out)


def train(net: ProposalNet, data: RenderedSet, epochs: int = 4, batch: int = 256, lr: float = 1e-3,
          lr_final: float = 5e-5, log=None):
    """Adam over the rendered set with fresh noise each epoch and a cosine
    learning-rate decay from lr to lr_final.  Returns the per-epoch mean loss."""
    if batch > net.max_batch:
        raise ValueError("batch exceeds the network's max_batch")
    px = data.side * data.side
    buf = torch.empty(batch * px, dtype=torch.float32, device=data.ctx.device)
    steps_per_epoch = data.n // batch
    total = max(1, epochs * steps_per_epoch)
    losses = []
    k = 0
    for ep in range(epochs):
        acc = torch.zeros(1, dtype=torch.float64, device=data.ctx.device)
        for s in range(steps_per_epoch):
            a = s * batch
            x = data.noisy(a, batch, ep, out=buf)
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * k / total))
            acc += net.train_step(x, data.targets[a:a + batch], rate)
            k += 1
        losses.append(float(acc.item()) / max(1, steps_per_epoch))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.5f}")
    return losses
