"""Tensor-level API over libgf (PyTorch-ROCm provides device memory and streams).

Every function validates shapes and dtypes on the host, hands raw device
pointers and sizes to the C ABI of ``include/gf.h`` on the current torch
stream, and returns torch tensors.  No step of the method runs in torch.

Parameter vectors: ``[x0, y0, Ie, Re, n, q, phi] * ncomp + [sky]`` per stamp,
flattened over the batch (``Batch.offsets['par']``).  Images are flattened
row-major per stamp at ``Batch.offsets['pix']`` (model, residual),
``['pad']`` (padded grids), ``['img']`` (data, weight) and ``['psf']``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L

GF_CONV_AUTO, GF_CONV_FFT, GF_CONV_DIRECT = L.GF_CONV_AUTO, L.GF_CONV_FFT, L.GF_CONV_DIRECT
GF_CONV_FFT_MULTIPASS, GF_CONV_FFT_FUSED = L.GF_CONV_FFT_MULTIPASS, L.GF_CONV_FFT_FUSED

LM_RESULT_DTYPE = np.dtype([("chi2", "<f8"), ("lambda", "<f8"), ("iters", "<i4"), ("nfev", "<i4"),
                            ("njev", "<i4"), ("status", "<i4"), ("reason", "<i4"), ("pad", "<i4")])


def _ptr(t):
    return 0 if t is None else int(t.data_ptr())


def _need(t, dtype, n, name):
    if t is None:
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    return t


class Context:
    """A libgf context bound to one HIP device; work goes on torch's current stream."""

    def __init__(self, device: int = 0, autotune_cache=None):
        """autotune_cache: path of the tuning file (None: no measuring, the
        default FFT-form rule)."""
        self.device = torch.device("cuda", device)
        self.ptr = L.gf_create(device, autotune_cache)

    def bind_stream(self):
        L.gf_set_stream(self.ptr, torch.cuda.current_stream(self.device).cuda_stream)

    def synchronize(self):
        L.gf_synchronize(self.ptr)

    def close(self):
        if getattr(self, "ptr", None):
            L.gf_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Stamp geometry of a batch (``gf_batch``)."""

    def __init__(self, ctx: Context, H, W, K, ncomp, shared: bool = False, group=None):
        self.ctx = ctx
        self.H, self.W, self.K, self.ncomp = list(map(int, H)), list(map(int, W)), list(map(int, K)), list(
            map(int, ncomp))
        self.n = len(self.H)
        self.shared = bool(shared)
        self.group = None if group is None else list(map(int, group))
        if self.group is not None:
            self.ptr = L.gf_batch_create_grouped(ctx.ptr, self.H, self.W, self.K, self.ncomp, self.group)
        else:
            self.ptr = L.gf_batch_create(ctx.ptr, self.H, self.W, self.K, self.ncomp, self.shared)
        self.n_groups = L.gf_batch_groups(self.ptr)
        self.sizes = L.gf_batch_sizes(self.ptr)
        self.offsets = L.gf_batch_offsets(self.ptr, self.n)
        self.P = [7 * c + 1 for c in self.ncomp]

    def close(self):
        if getattr(self, "ptr", None):
            L.gf_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Psf:
    """Prepared PSFs of a batch (``gf_psf``); keeps the taps tensor alive."""

    def __init__(self, ctx: Context, batch: Batch, taps: torch.Tensor, mode: int = GF_CONV_AUTO):
        _need(taps, torch.float32, batch.sizes["n_psf"], "taps")
        self.ctx, self.batch, self.taps = ctx, batch, taps
        ctx.bind_stream()
        self.ptr = L.gf_psf_prepare(ctx.ptr, batch.ptr, _ptr(taps), int(mode))
        self.uses_fft, self.fft_side = L.gf_psf_paths(self.ptr, batch.n)

    def close(self):
        if getattr(self, "ptr", None):
            L.gf_psf_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _empty(ctx, n, dtype=torch.float32):
    return torch.empty(int(max(n, 1)), dtype=dtype, device=ctx.device)


def eval_model(ctx: Context, batch: Batch, theta: torch.Tensor, oversample: int = 5, out=None) -> torch.Tensor:
    """Step 1 (gf_eval_model): padded model grids, no sky, flat [n_pad]."""
    _need(theta, torch.float32, batch.sizes["n_par"], "theta")
    out = _empty(ctx, batch.sizes["n_pad"]) if out is None else _need(out, torch.float32, batch.sizes["n_pad"], "out")
    ctx.bind_stream()
    L.gf_eval_model(ctx.ptr, batch.ptr, _ptr(theta), int(oversample), _ptr(out))
    return out


def convolve_psf(ctx: Context, batch: Batch, psf: Psf, model_pad: torch.Tensor, n_ch: int = 1, out=None):
    """Step 2 (gf_convolve_psf): valid convolution, flat [n_pix * n_ch]."""
    _need(model_pad, torch.float32, batch.sizes["n_pad"] * n_ch, "model_pad")
    n = batch.sizes["n_pix"] * n_ch
    out = _empty(ctx, n) if out is None else _need(out, torch.float32, n, "out")
    ctx.bind_stream()
    L.gf_convolve_psf(ctx.ptr, batch.ptr, psf.ptr, _ptr(model_pad), int(n_ch), _ptr(out))
    return out


def model(ctx: Context, batch: Batch, psf: Psf, theta: torch.Tensor, oversample: int = 5, out=None):
    """Steps 1-2 plus sky (gf_model): flat [n_pix]."""
    _need(theta, torch.float32, batch.sizes["n_par"], "theta")
    out = _empty(ctx, batch.sizes["n_pix"]) if out is None else _need(out, torch.float32, batch.sizes["n_pix"], "out")
    ctx.bind_stream()
    L.gf_model(ctx.ptr, batch.ptr, psf.ptr, _ptr(theta), int(oversample), _ptr(out), 0)
    return out


def chi2(ctx: Context, batch: Batch, model_img: torch.Tensor, theta: torch.Tensor, data: torch.Tensor,
         weight: torch.Tensor, want_resid: bool = False):
    """Step 3 (gf_chi2).  Returns (pairs [n, 2] FP32 (hi, lo), resid or None)."""
    _need(model_img, torch.float32, batch.sizes["n_pix"], "model")
    _need(theta, torch.float32, batch.sizes["n_par"], "theta")
    _need(data, torch.float32, batch.sizes["n_img"], "data")
    _need(weight, torch.float32, batch.sizes["n_img"], "weight")
    pairs = torch.empty((batch.n, 2), dtype=torch.float32, device=ctx.device)
    resid = _empty(ctx, batch.sizes["n_pix"]) if want_resid else None
    ctx.bind_stream()
    L.gf_chi2(ctx.ptr, batch.ptr, _ptr(model_img), _ptr(theta), _ptr(data), _ptr(weight), _ptr(resid), _ptr(pairs))
    return pairs, resid


def chi2_noalloc(ctx: Context, batch: Batch, model_img: torch.Tensor, theta: torch.Tensor, data: torch.Tensor,
                 weight: torch.Tensor, want_resid: bool = False, out=None, resid=None):
    """Step 3 without any library allocation (gf_chi2_noalloc): the same
    result as chi2().  Returns (pairs [n, 2] FP32 (hi, lo), resid or None)."""
    _need(model_img, torch.float32, batch.sizes["n_pix"], "model")
    _need(theta, torch.float32, batch.sizes["n_par"], "theta")
    _need(data, torch.float32, batch.sizes["n_img"], "data")
    _need(weight, torch.float32, batch.sizes["n_img"], "weight")
    pairs = torch.empty((batch.n, 2), dtype=torch.float32, device=ctx.device) if out is None else out
    if want_resid and resid is None:
        resid = _empty(ctx, batch.sizes["n_pix"])
    ctx.bind_stream()
    L.gf_chi2_noalloc(ctx.ptr, batch.ptr, _ptr(model_img), _ptr(theta), _ptr(data), _ptr(weight),
                      _ptr(resid if want_resid else None), _ptr(pairs))
    return pairs, (resid if want_resid else None)


def pairs_to_f64(pairs: torch.Tensor) -> torch.Tensor:
    """Unpack (hi, lo) FP32 pairs into the FP64 values they represent."""
    return pairs[:, 0].double() + pairs[:, 1].double()


def likelihood(ctx: Context, batch: Batch, psf: Psf, theta: torch.Tensor, data: torch.Tensor, weight: torch.Tensor,
               oversample: int = 5, work=None, out=None) -> torch.Tensor:
    """Steps 1-3 in one call (gf_likelihood): (hi, lo) chi2 pairs [n, 2]."""
    _need(theta, torch.float32, batch.sizes["n_par"], "theta")
    _need(data, torch.float32, batch.sizes["n_img"], "data")
    _need(weight, torch.float32, batch.sizes["n_img"], "weight")
    out = torch.empty((batch.n, 2), dtype=torch.float32, device=ctx.device) if out is None else out
    ctx.bind_stream()
    L.gf_likelihood(ctx.ptr, batch.ptr, psf.ptr, _ptr(theta), int(oversample), _ptr(data), _ptr(weight), _ptr(out),
                    _ptr(work))
    return out


def likelihood_workspace(ctx: Context, batch: Batch, psf: Psf) -> torch.Tensor:
    n = L.gf_likelihood_workspace(batch.ptr, psf.ptr)
    return torch.empty(int(n), dtype=torch.uint8, device=ctx.device)


def jacobian_full(ctx: Context, batch: Batch, psf: Psf, theta: torch.Tensor, oversample: int = 5, out=None):
    """d m / d theta images (gf_jacobian, GF_JAC_FULL), flat [n_jac]."""
    _need(theta, torch.float32, batch.sizes["n_par"], "theta")
    out = _empty(ctx, batch.sizes["n_jac"]) if out is None else _need(out, torch.float32, batch.sizes["n_jac"], "out")
    ctx.bind_stream()
    L.gf_jacobian(ctx.ptr, batch.ptr, psf.ptr, _ptr(theta), int(oversample), L.GF_JAC_FULL, 0, 0, 1.0, _ptr(out))
    return out


def jacobian_adjoint(ctx: Context, batch: Batch, psf: Psf, theta: torch.Tensor, cot: torch.Tensor, weight=None,
                     scale: float = 1.0, oversample: int = 5, out=None):
    """scale * sum_i cot_i (sqrt(w_i)) d m_i / d theta (gf_jacobian, GF_JAC_ADJOINT), flat [n_par]."""
    _need(theta, torch.float32, batch.sizes["n_par"], "theta")
    _need(cot, torch.float32, batch.sizes["n_pix"], "cot")
    if weight is not None:
        _need(weight, torch.float32, batch.sizes["n_img"], "weight")
    out = _empty(ctx, batch.sizes["n_par"]) if out is None else _need(out, torch.float32, batch.sizes["n_par"], "out")
    ctx.bind_stream()
    L.gf_jacobian(ctx.ptr, batch.ptr, psf.ptr, _ptr(theta), int(oversample), L.GF_JAC_ADJOINT, _ptr(cot),
                  _ptr(weight), float(scale), _ptr(out))
    return out


def lm_options(**kw) -> L.GfLmOpts:
    o = L.gf_lm_opts_default()
    for k, v in kw.items():
        if k in ("lo", "hi", "free_mask"):
            continue
        if k == "lambda_":
            k = "lambda0"
        setattr(o, k, v)
    return o


def fit_lm(ctx: Context, batch: Batch, psf: Psf, data: torch.Tensor, weight: torch.Tensor, theta0: torch.Tensor,
           lo=None, hi=None, free=None, return_device=False, **opts):
    """Levenberg-Marquardt over the whole batch on the device (gf_fit_lm).

    theta0: float64 device tensor [n_par] (not modified).  Returns
    (theta float64 tensor, numpy structured array of per-stamp results)."""
    n_par = batch.sizes["n_par"]
    _need(theta0, torch.float64, n_par, "theta0")
    _need(data, torch.float32, batch.sizes["n_img"], "data")
    _need(weight, torch.float32, batch.sizes["n_img"], "weight")
    o = lm_options(**opts)
    if lo is not None:
        o.lo = _ptr(_need(lo, torch.float64, n_par, "lo"))
    if hi is not None:
        o.hi = _ptr(_need(hi, torch.float64, n_par, "hi"))
    if free is not None:
        o.free_mask = _ptr(_need(free, torch.uint8, n_par, "free"))
    # the library reads the start from theta0 and writes the fit to theta
    o.start = _ptr(theta0)
    theta = torch.empty_like(theta0)
    if theta0.numel() > n_par:
        theta[n_par:].copy_(theta0[n_par:])
    res = torch.empty(batch.n * LM_RESULT_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)
    ctx.bind_stream()
    L.gf_fit_lm(ctx.ptr, batch.ptr, psf.ptr, _ptr(data), _ptr(weight), _ptr(theta), o, _ptr(res))
    if return_device:
        return theta, res
    info = np.frombuffer(res.cpu().numpy().tobytes(), dtype=LM_RESULT_DTYPE)
    return theta, info


def lm_info(res: torch.Tensor):
    """Per-stamp results (numpy structured array) from the device records."""
    return np.frombuffer(res.cpu().numpy().tobytes(), dtype=LM_RESULT_DTYPE)


def group_best(ctx: Context, batch: Batch, res: torch.Tensor, theta: torch.Tensor):
    """Lowest-chi^2 member per observation group (gf_group_best): (best
    parameters float64 [n_groups, 29], winning stamp int32 [n_groups])."""
    _need(theta, torch.float64, batch.sizes["n_par"], "theta")
    best = torch.empty((batch.n_groups, 29), dtype=torch.float64, device=ctx.device)
    idx = torch.empty(batch.n_groups, dtype=torch.int32, device=ctx.device)
    ctx.bind_stream()
    L.gf_group_best(ctx.ptr, batch.ptr, _ptr(res), _ptr(theta), _ptr(best), _ptr(idx))
    return best, idx


def expand_starts(ctx: Context, theta0: torch.Tensor, n_starts: int) -> torch.Tensor:
    """Multi-start set [n_groups * n_starts, 8] (gf_expand_starts)."""
    G = theta0.numel() // 8
    _need(theta0, torch.float64, G * 8, "theta0")
    out = torch.empty((max(G * n_starts, 1), 8), dtype=torch.float64, device=ctx.device)
    ctx.bind_stream()
    L.gf_expand_starts(ctx.ptr, G, int(n_starts), _ptr(theta0), _ptr(out))
    return out[:G * n_starts]


# ------------------------------------------------------------ spectral lines
class LineBatch:
    """Spectra of a line batch (``gf_line_batch``): N channels, K LSF taps and
    1..3 Gaussian lines each.  Parameters per spectrum ``[A, mu, sigma] *
    n_lines + [continuum]``; flat offsets in ``offsets['data'|'lsf'|'par']``."""

    def __init__(self, ctx: Context, N, K, n_lines):
        self.ctx = ctx
        self.n = len(N)
        self.ptr = L.gf_line_batch_create(ctx.ptr, N, K, n_lines)
        self.offsets = L.gf_line_batch_offsets(self.ptr, self.n)
        self.sizes = {k: int(v[-1]) for k, v in self.offsets.items()}

    def close(self):
        if getattr(self, "ptr", None):
            L.gf_line_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def line_model(ctx: Context, lb: LineBatch, lsf: torch.Tensor, theta: torch.Tensor, oversample: int = 5,
               out=None) -> torch.Tensor:
    """Model spectra (gf_line_model), flat [n_data] float32."""
    _need(lsf, torch.float32, lb.sizes["lsf"], "lsf")
    _need(theta, torch.float32, lb.sizes["par"], "theta")
    out = _empty(ctx, lb.sizes["data"]) if out is None else _need(out, torch.float32, lb.sizes["data"], "out")
    ctx.bind_stream()
    L.gf_line_model(ctx.ptr, lb.ptr, _ptr(lsf), _ptr(theta), int(oversample), _ptr(out))
    return out


def line_chi2(ctx: Context, lb: LineBatch, lsf: torch.Tensor, theta: torch.Tensor, data: torch.Tensor,
              weight: torch.Tensor, oversample: int = 5) -> torch.Tensor:
    """chi^2 (hi, lo) pairs [n, 2] of every spectrum (gf_line_chi2)."""
    _need(lsf, torch.float32, lb.sizes["lsf"], "lsf")
    _need(theta, torch.float32, lb.sizes["par"], "theta")
    _need(data, torch.float32, lb.sizes["data"], "data")
    _need(weight, torch.float32, lb.sizes["data"], "weight")
    out = torch.empty((lb.n, 2), dtype=torch.float32, device=ctx.device)
    ctx.bind_stream()
    L.gf_line_chi2(ctx.ptr, lb.ptr, _ptr(lsf), _ptr(theta), int(oversample), _ptr(data), _ptr(weight), _ptr(out))
    return out


def line_fit_lm(ctx: Context, lb: LineBatch, lsf: torch.Tensor, data: torch.Tensor, weight: torch.Tensor,
                theta0: torch.Tensor, lo=None, hi=None, free=None, return_device=False, **opts):
    """Levenberg-Marquardt over every spectrum (gf_line_fit_lm), one
    workgroup per spectrum in one launch.  theta0: float64 [n_par] (not
    modified).  Returns (theta, per-spectrum results) as fit_lm does."""
    n_par = lb.sizes["par"]
    _need(lsf, torch.float32, lb.sizes["lsf"], "lsf")
    _need(theta0, torch.float64, n_par, "theta0")
    _need(data, torch.float32, lb.sizes["data"], "data")
    _need(weight, torch.float32, lb.sizes["data"], "weight")
    o = lm_options(**opts)
    if lo is not None:
        o.lo = _ptr(_need(lo, torch.float64, n_par, "lo"))
    if hi is not None:
        o.hi = _ptr(_need(hi, torch.float64, n_par, "hi"))
    if free is not None:
        o.free_mask = _ptr(_need(free, torch.uint8, n_par, "free"))
    theta = theta0.clone()
    res = torch.empty(lb.n * LM_RESULT_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)
    ctx.bind_stream()
    L.gf_line_fit_lm(ctx.ptr, lb.ptr, _ptr(lsf), _ptr(data), _ptr(weight), _ptr(theta), o, _ptr(res))
    if return_device:
        return theta, res
    return theta, lm_info(res)


class CubeBatch:
    """Data cubes (``gf_cube_batch``): n cubes of Nc channels of an H x W
    image with a K x K PSF each, one LSF length for the batch.  Parameters
    per cube ``[xc, yc, Ie, Re, n, q, phi, continuum, v0, vproj, rt,
    sigma_v]`` (FP64); flat offsets in ``offsets['vox'|'psf'|'lsf'|'par']``.
    ``set_kernels`` must run before the model, chi^2, Jacobian and fit."""

    def __init__(self, ctx: Context, H, W, K, n_chan: int, k_lsf: int):
        self.ctx = ctx
        self.n = len(H)
        self.n_chan, self.k_lsf = int(n_chan), int(k_lsf)
        self.ptr = L.gf_cube_batch_create(ctx.ptr, H, W, K, n_chan, k_lsf)
        self.offsets = L.gf_cube_batch_offsets(self.ptr, self.n)
        self.sizes = {k: int(v[-1]) for k, v in self.offsets.items()}

    def set_kernels(self, psf: torch.Tensor, lsf: torch.Tensor, mode: int = GF_CONV_AUTO):
        _need(psf, torch.float32, self.sizes["psf"], "psf")
        _need(lsf, torch.float32, self.sizes["lsf"], "lsf")
        self.ctx.bind_stream()
        L.gf_cube_set_kernels(self.ctx.ptr, self.ptr, _ptr(psf), _ptr(lsf), int(mode))

    def close(self):
        if getattr(self, "ptr", None):
            L.gf_cube_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cube_model(ctx: Context, cb: CubeBatch, theta: torch.Tensor, oversample: int = 5, oversample_v: int = 3,
               out=None) -> torch.Tensor:
    """Model cubes (gf_cube_model), flat [n_vox] float32."""
    _need(theta, torch.float64, cb.sizes["par"], "theta")
    out = _empty(ctx, cb.sizes["vox"]) if out is None else _need(out, torch.float32, cb.sizes["vox"], "out")
    ctx.bind_stream()
    L.gf_cube_model(ctx.ptr, cb.ptr, _ptr(theta), int(oversample), int(oversample_v), _ptr(out))
    return out


def cube_chi2(ctx: Context, cb: CubeBatch, theta: torch.Tensor, data: torch.Tensor, weight: torch.Tensor,
              oversample: int = 5, oversample_v: int = 3) -> torch.Tensor:
    """chi^2 (hi, lo) pairs [n, 2] of every cube (gf_cube_chi2)."""
    _need(theta, torch.float64, cb.sizes["par"], "theta")
    _need(data, torch.float32, cb.sizes["vox"], "data")
    _need(weight, torch.float32, cb.sizes["vox"], "weight")
    out = torch.empty((cb.n, 2), dtype=torch.float32, device=ctx.device)
    ctx.bind_stream()
    L.gf_cube_chi2(ctx.ptr, cb.ptr, _ptr(theta), int(oversample), int(oversample_v), _ptr(data), _ptr(weight),
                   _ptr(out))
    return out


def cube_jacobian(ctx: Context, cb: CubeBatch, theta: torch.Tensor, oversample: int = 5,
                  oversample_v: int = 3) -> torch.Tensor:
    """d model / d theta (gf_cube_jacobian), flat [12 n_vox] float32: cube s's
    12 derivative cubes from 12 * offsets['vox'][s]."""
    _need(theta, torch.float64, cb.sizes["par"], "theta")
    out = _empty(ctx, L.GF_CUBE_NPAR * cb.sizes["vox"])
    ctx.bind_stream()
    L.gf_cube_jacobian(ctx.ptr, cb.ptr, _ptr(theta), int(oversample), int(oversample_v), _ptr(out))
    return out


def cube_fit_lm(ctx: Context, cb: CubeBatch, data: torch.Tensor, weight: torch.Tensor, theta0: torch.Tensor,
                oversample_v: int = 3, lo=None, hi=None, free=None, return_device=False, **opts):
    """Levenberg-Marquardt over every cube (gf_cube_fit_lm).  theta0: float64
    [n_par] (not modified).  Returns (theta, per-cube results) as fit_lm does."""
    n_par = cb.sizes["par"]
    _need(theta0, torch.float64, n_par, "theta0")
    _need(data, torch.float32, cb.sizes["vox"], "data")
    _need(weight, torch.float32, cb.sizes["vox"], "weight")
    o = lm_options(**opts)
    if lo is not None:
        o.lo = _ptr(_need(lo, torch.float64, n_par, "lo"))
    if hi is not None:
        o.hi = _ptr(_need(hi, torch.float64, n_par, "hi"))
    if free is not None:
        o.free_mask = _ptr(_need(free, torch.uint8, n_par, "free"))
    theta = theta0.clone()
    res = torch.empty(cb.n * LM_RESULT_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)
    ctx.bind_stream()
    L.gf_cube_fit_lm(ctx.ptr, cb.ptr, _ptr(data), _ptr(weight), _ptr(theta), o, int(oversample_v), _ptr(res))
    if return_device:
        return theta, res
    return theta, lm_info(res)


# ------------------------------------------------------------------ autograd
class Chi2Fn(torch.autograd.Function):
    """chi^2 per stamp (FP64 from the compensated pair) with the adjoint
    gradient d chi^2 / d theta = -2 sum_i sqrt(w_i) r_i d m_i / d theta."""

    @staticmethod
    def forward(fctx, theta, ctx, batch, psf, data, weight, oversample):
        mp = eval_model(ctx, batch, theta, oversample)
        m = convolve_psf(ctx, batch, psf, mp)
        pairs, resid = chi2(ctx, batch, m, theta, data, weight, want_resid=True)
        fctx.save_for_backward(theta, resid, weight)
        fctx.gf = (ctx, batch, psf, oversample)
        return pairs_to_f64(pairs)

    @staticmethod
    def backward(fctx, g):
        theta, resid, weight = fctx.saved_tensors
        ctx, batch, psf, oversample = fctx.gf
        grad = jacobian_adjoint(ctx, batch, psf, theta, resid, weight, -2.0, oversample)
        per = torch.repeat_interleave(g.to(torch.float32), torch.tensor(batch.P, device=g.device))
        return grad * per, None, None, None, None, None, None


class ModelFn(torch.autograd.Function):
    """Model image conv(components) + sky with the vector-Jacobian product
    computed by the adjoint kernels."""

    @staticmethod
    def forward(fctx, theta, ctx, batch, psf, oversample):
        fctx.save_for_backward(theta)
        fctx.gf = (ctx, batch, psf, oversample)
        return model(ctx, batch, psf, theta, oversample)

    @staticmethod
    def backward(fctx, g):
        (theta,) = fctx.saved_tensors
        ctx, batch, psf, oversample = fctx.gf
        return jacobian_adjoint(ctx, batch, psf, theta, g.contiguous().to(torch.float32), None, 1.0,
                                oversample), None, None, None, None


# ------------------------------------------------------------------ MCMC
def mcmc_run(ctx: Context, batch: Batch, psf: Psf, data: torch.Tensor, weight: torch.Tensor, theta0: torch.Tensor,
             scale: torch.Tensor, n_steps: int, key=(0, 0), stream: int = 0, step0: int = 0, thin: int = 1,
             lo=None, hi=None, keep_samples: bool = True, oversample: int = 5, use_graph: bool = True):
    """Random-walk Metropolis, one chain per stamp (gf_mcmc_run).

    Returns (theta float64 [n_par] after the last step, chi2 float64 [n],
    samples float32 [n_steps // thin, n_par] or None, accepted int32 [n])."""
    n_par = batch.sizes["n_par"]
    _need(theta0, torch.float64, n_par, "theta0")
    _need(scale, torch.float64, n_par, "scale")
    _need(data, torch.float32, batch.sizes["n_img"], "data")
    _need(weight, torch.float32, batch.sizes["n_img"], "weight")
    o = L.gf_mcmc_opts_default()
    o.n_steps, o.oversample, o.thin, o.use_graph = int(n_steps), int(oversample), int(thin), int(bool(use_graph))
    o.key0, o.key1, o.stream, o.step0 = int(key[0]), int(key[1]), int(stream), int(step0)
    o.scale = _ptr(scale)
    if lo is not None:
        o.lo = _ptr(_need(lo, torch.float64, n_par, "lo"))
    if hi is not None:
        o.hi = _ptr(_need(hi, torch.float64, n_par, "hi"))
    theta = theta0.clone()
    chi2v = torch.empty(batch.n, dtype=torch.float64, device=ctx.device)
    nk = int(n_steps) // int(thin)
    samples = torch.empty((max(nk, 1), n_par), dtype=torch.float32, device=ctx.device) if keep_samples else None
    acc = torch.zeros(batch.n, dtype=torch.int32, device=ctx.device)
    ctx.bind_stream()
    L.gf_mcmc_run(ctx.ptr, batch.ptr, psf.ptr, _ptr(data), _ptr(weight), _ptr(theta), _ptr(chi2v), o,
                  _ptr(samples), _ptr(acc))
    return theta, chi2v, (samples[:nk] if samples is not None else None), acc


# ------------------------------------------------------------------ downhill simplex
def fit_simplex(ctx: Context, batch: Batch, psf: Psf, data: torch.Tensor, weight: torch.Tensor,
                theta0: torch.Tensor, step: torch.Tensor, lo=None, hi=None, max_iter: int = 2000, ftol: float = 1e-8,
                oversample: int = 5, poll_every: int = 16, use_graph: bool = True, trace_cap: int = 0):
    """Nelder-Mead over the whole batch on the device (gf_fit_simplex).

    Returns (theta float64 [n_par], per-stamp results as for fit_lm, trace
    float64 [n_stamps, trace_cap] of evaluated chi^2 values or None)."""
    n_par = batch.sizes["n_par"]
    _need(theta0, torch.float64, n_par, "theta0")
    _need(step, torch.float64, n_par, "step")
    _need(data, torch.float32, batch.sizes["n_img"], "data")
    _need(weight, torch.float32, batch.sizes["n_img"], "weight")
    o = L.gf_simplex_opts_default()
    o.max_iter, o.oversample, o.ftol = int(max_iter), int(oversample), float(ftol)
    o.poll_every, o.use_graph = int(poll_every), int(bool(use_graph))
    o.step = _ptr(step)
    if lo is not None:
        o.lo = _ptr(_need(lo, torch.float64, n_par, "lo"))
    if hi is not None:
        o.hi = _ptr(_need(hi, torch.float64, n_par, "hi"))
    theta = theta0.clone()
    res = torch.empty(batch.n * LM_RESULT_DTYPE.itemsize, dtype=torch.uint8, device=ctx.device)
    trace = torch.full((batch.n, trace_cap), float("nan"), dtype=torch.float64, device=ctx.device) if trace_cap else None
    ctx.bind_stream()
    L.gf_fit_simplex(ctx.ptr, batch.ptr, psf.ptr, _ptr(data), _ptr(weight), _ptr(theta), o, _ptr(res), _ptr(trace),
                     int(trace_cap))
    return theta, lm_info(res), trace
