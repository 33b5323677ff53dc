"""Shared set-up of the GPU parity tests: batches of synthetic stamps run
through the C ABI, and the same FP32 inputs handed to the FP64 oracle."""
from __future__ import annotations

import numpy as np
import torch

from paper_1101_2254_amd import ops


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda", 0)


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev(), dtype=dtype)


class GpuBatch:
    """A batch of stamps with FP32 parameters, PSFs, data and weights on the
    device, plus the float64 copies of the same FP32 values for the oracle."""

    def __init__(self, ctx, stamps, thetas=None, data=None, weights=None, mode=ops.GF_CONV_AUTO, shared=False):
        self.ctx = ctx
        self.stamps = stamps
        n = len(stamps)
        H = [s.H for s in stamps]
        W = [s.W for s in stamps]
        K = [s.K for s in stamps]
        nc = [s.ncomp for s in stamps]
        self.batch = ops.Batch(ctx, H, W, K, nc, shared)
        if thetas is None:
            thetas = [s.truth for s in stamps]
        self.th32 = [np.asarray(t, np.float32) for t in thetas]
        self.psf32 = [s.psf.astype(np.float32) for s in (stamps[:1] if shared else stamps)]
        self.theta = to_dev(np.concatenate(self.th32))
        self.taps = to_dev(np.concatenate([p.ravel() for p in self.psf32]))
        self.psf = ops.Psf(ctx, self.batch, self.taps, mode)
        if data is not None:
            self.d32 = [np.asarray(x, np.float32) for x in data]
            self.w32 = [np.asarray(x, np.float32) for x in weights]
            self.data = to_dev(np.concatenate([x.ravel() for x in self.d32]))
            self.weight = to_dev(np.concatenate([x.ravel() for x in self.w32]))
        self.n = n

    def th64(self, s):
        return self.th32[s].astype(np.float64)

    def psf64(self, s):
        return self.psf32[0 if self.batch.shared else s].astype(np.float64)

    def split_pix(self, flat, n_ch=1):
        out = []
        f = flat.detach().cpu().numpy()
        for s, st in enumerate(self.stamps):
            o = self.batch.offsets["pix"][s] * n_ch
            out.append(f[o:o + n_ch * st.H * st.W].reshape(n_ch, st.H, st.W) if n_ch > 1 else
                       f[o:o + st.H * st.W].reshape(st.H, st.W))
        return out

    def split_pad(self, flat, n_ch=1):
        out = []
        f = flat.detach().cpu().numpy()
        for s, st in enumerate(self.stamps):
            Mh, Mw = st.H + st.K - 1, st.W + st.K - 1
            o = self.batch.offsets["pad"][s] * n_ch
            out.append(f[o:o + n_ch * Mh * Mw].reshape(n_ch, Mh, Mw) if n_ch > 1 else
                       f[o:o + Mh * Mw].reshape(Mh, Mw))
        return out


def keep_fft_forms(ctx):
    """Keep one-workgroup stamps on that form to the end of every fit (no
    move to the multi-pass launches when few remain), so a stamp's fit does
    not depend on how many other stamps of its batch are still fitting:
    the bitwise batch-independence checks rely on it."""
    from paper_1101_2254_amd import _lib as L
    for side in (64, 96, 128, 160, 192):
        L.gf_tune_min_active_set(ctx.ptr, side, 0)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))
