"""ctypes binding of ``libgf.so`` (declared in ``include/gf.h``).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Importing this module does not touch the GPU; :func:`lib` loads the
library and raises if it has not been built, so no call can fall back to
anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgf.so")

GF_OK, GF_EINVAL, GF_ESHAPE, GF_ENOMEM, GF_EDEVICE, GF_ENUMERIC, GF_ENOTCONV = range(7)
STATUS_NAMES = {0: "GF_OK", 1: "GF_EINVAL", 2: "GF_ESHAPE", 3: "GF_ENOMEM", 4: "GF_EDEVICE", 5: "GF_ENUMERIC",
                6: "GF_ENOTCONV"}
GF_NPC = 7
GF_MAX_COMP = 4
GF_CONV_AUTO, GF_CONV_FFT, GF_CONV_DIRECT, GF_CONV_FFT_MULTIPASS, GF_CONV_FFT_FUSED = 0, 1, 2, 3, 4
GF_FFT_FUSED_MAX = 192
GF_JAC_FULL, GF_JAC_ADJOINT = 0, 1
GF_CUBE_NPAR = 12
GF_CUBE_MAX_CHAN = 1024

# Every symbol that include/gf.h declares.
EXPORTS = ("gf_create", "gf_destroy", "gf_set_stream", "gf_last_error", "gf_synchronize", "gf_batch_create",
           "gf_batch_destroy", "gf_batch_create_grouped", "gf_batch_groups", "gf_group_best", "gf_expand_starts", "gf_batch_sizes", "gf_batch_offsets", "gf_batch_count", "gf_psf_prepare",
           "gf_psf_destroy", "gf_psf_paths", "gf_eval_model", "gf_convolve_psf", "gf_model", "gf_chi2", "gf_likelihood",
           "gf_likelihood_workspace", "gf_jacobian", "gf_lm_opts_default", "gf_fit_lm", "gf_mcmc_opts_default", "gf_mcmc_run",
           "gf_simplex_opts_default", "gf_fit_simplex",
           "gf_moments_guess",
           "gf_cnn_create", "gf_cnn_destroy", "gf_cnn_param_count", "gf_cnn_init", "gf_cnn_set_params",
           "gf_cnn_get_params", "gf_cnn_forward", "gf_cnn_gradients", "gf_cnn_train_step", "gf_cnn_steps",
           "gf_cnn_encode", "gf_cnn_decode", "gf_philox", "gf_normal_noise", "gf_draw_prior", "gf_probe", "gf_profile_start",
           "gf_profile_stop", "gf_profile_kernels", "gf_profile_get", "gf_line_batch_create", "gf_line_batch_destroy",
           "gf_line_batch_offsets", "gf_line_model", "gf_line_chi2", "gf_line_fit_lm", "gf_version",
           "gf_chi2_noalloc", "gf_autotune", "gf_tune_form_get", "gf_tune_form_set", "gf_tune_min_active_get", "gf_tune_min_active_set",
           "gf_tune_direct_get", "gf_tune_direct_set",
           "gf_cube_batch_create", "gf_cube_batch_destroy", "gf_cube_batch_offsets", "gf_cube_set_kernels",
           "gf_cube_model", "gf_cube_chi2", "gf_cube_jacobian", "gf_cube_fit_lm")


class GfLmOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("lambda0", ctypes.c_double),
                ("lambda_up", ctypes.c_double), ("lambda_down", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("ftol", ctypes.c_double), ("xtol", ctypes.c_double),
                ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p), ("free_mask", ctypes.c_void_p),
                ("poll_every", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("speculate", ctypes.c_int32),
                ("start", ctypes.c_void_p)]


class GfMcmcOpts(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("oversample", ctypes.c_int32), ("thin", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("key0", ctypes.c_uint64), ("key1", ctypes.c_uint64),
                ("stream", ctypes.c_uint64), ("step0", ctypes.c_int64), ("scale", ctypes.c_void_p),
                ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p)]


class GfSimplexOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("oversample", ctypes.c_int32), ("ftol", ctypes.c_double),
                ("step", ctypes.c_void_p), ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p),
                ("poll_every", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class GfLmResult(ctypes.Structure):
    _fields_ = [("chi2", ctypes.c_double), ("lambda_", ctypes.c_double), ("iters", ctypes.c_int32),
                ("nfev", ctypes.c_int32), ("njev", ctypes.c_int32), ("status", ctypes.c_int32),
                ("reason", ctypes.c_int32), ("pad", ctypes.c_int32)]


_lib = None


class GfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """Load libgf.so (built by ``paper_1101_2254_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1101_2254_amd.build` "
                           "(there is no other implementation to fall back to)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, flt = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    u64 = ctypes.c_uint64
    pvp = ctypes.POINTER(ctypes.c_void_p)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "gf_create": (i32, [pvp, i32, ctypes.c_char_p]),
        "gf_autotune": (i32, [vp, vp, i32]),
        "gf_chi2_noalloc": (i32, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "gf_destroy": (None, [vp]),
        "gf_set_stream": (i32, [vp, vp]),
        "gf_last_error": (ctypes.c_char_p, [vp]),
        "gf_synchronize": (i32, [vp]),
        "gf_batch_create": (i32, [vp, i32, vp, vp, vp, vp, i32, pvp]),
        "gf_batch_destroy": (None, [vp]),
        "gf_batch_create_grouped": (i32, [vp, i32, vp, vp, vp, vp, vp, pvp]),
        "gf_batch_groups": (i32, [vp]),
        "gf_group_best": (i32, [vp, vp, vp, vp, vp, vp]),
        "gf_expand_starts": (i32, [vp, i32, i32, vp, vp]),
        "gf_batch_sizes": (i32, [vp, pi64, pi64, pi64, pi64, pi64, pi64]),
        "gf_batch_offsets": (i32, [vp, vp, vp, vp, vp, vp, vp]),
        "gf_batch_count": (i32, [vp]),
        "gf_psf_prepare": (i32, [vp, vp, vp, i32, pvp]),
        "gf_psf_destroy": (None, [vp]),
        "gf_psf_paths": (i32, [vp, vp, vp]),
        "gf_eval_model": (i32, [vp, vp, vp, i32, vp]),
        "gf_convolve_psf": (i32, [vp, vp, vp, vp, i32, vp]),
        "gf_model": (i32, [vp, vp, vp, vp, i32, vp, vp]),
        "gf_chi2": (i32, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "gf_likelihood": (i32, [vp, vp, vp, vp, i32, vp, vp, vp, vp]),
        "gf_likelihood_workspace": (i64, [vp, vp]),
        "gf_jacobian": (i32, [vp, vp, vp, vp, i32, i32, vp, vp, flt, vp]),
        "gf_lm_opts_default": (None, [ctypes.POINTER(GfLmOpts)]),
        "gf_fit_lm": (i32, [vp, vp, vp, vp, vp, vp, ctypes.POINTER(GfLmOpts), vp]),
        "gf_mcmc_opts_default": (None, [ctypes.POINTER(GfMcmcOpts)]),
        "gf_mcmc_run": (i32, [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(GfMcmcOpts), vp, vp]),
        "gf_simplex_opts_default": (None, [ctypes.POINTER(GfSimplexOpts)]),
        "gf_fit_simplex": (i32, [vp, vp, vp, vp, vp, vp, ctypes.POINTER(GfSimplexOpts), vp, vp, i32]),
        "gf_moments_guess": (i32, [vp, vp, vp, vp]),
        "gf_cnn_create": (i32, [vp, i32, i32, pvp]),
        "gf_cnn_destroy": (None, [vp]),
        "gf_cnn_param_count": (i64, [vp]),
        "gf_cnn_init": (i32, [vp, u64]),
        "gf_cnn_set_params": (i32, [vp, vp]),
        "gf_cnn_get_params": (i32, [vp, vp]),
        "gf_cnn_forward": (i32, [vp, vp, i32, vp]),
        "gf_cnn_gradients": (i32, [vp, vp, vp, i32, vp, vp]),
        "gf_cnn_train_step": (i32, [vp, vp, vp, i32, flt, vp]),
        "gf_cnn_steps": (i64, [vp]),
        "gf_cnn_encode": (i32, [vp, i32, i32, vp, vp]),
        "gf_cnn_decode": (i32, [vp, i32, i32, vp, vp]),
        "gf_philox": (i32, [vp, u64, u64, vp, i64, vp]),
        "gf_normal_noise": (i32, [vp, i64, flt, u64, u64, vp, vp, vp]),
        "gf_draw_prior": (i32, [vp, i32, i32, u64, u64, vp, vp]),
        "gf_probe": (i32, [vp, i32, i64, i32, ctypes.POINTER(ctypes.c_double)]),
        "gf_profile_start": (i32, [vp]),
        "gf_profile_stop": (i32, [vp]),
        "gf_profile_kernels": (i32, [vp]),
        "gf_profile_get": (i32, [vp, i32, ctypes.c_char_p, i32, pi64, ctypes.POINTER(ctypes.c_double)]),
        "gf_line_batch_create": (i32, [vp, i32, vp, vp, vp, pvp]),
        "gf_line_batch_destroy": (None, [vp]),
        "gf_line_batch_offsets": (i32, [vp, vp, vp, vp]),
        "gf_line_model": (i32, [vp, vp, vp, vp, i32, vp]),
        "gf_line_chi2": (i32, [vp, vp, vp, vp, i32, vp, vp, vp]),
        "gf_line_fit_lm": (i32, [vp, vp, vp, vp, vp, vp, ctypes.POINTER(GfLmOpts), vp]),
        "gf_cube_batch_create": (i32, [vp, i32, vp, vp, vp, i32, i32, pvp]),
        "gf_cube_batch_destroy": (None, [vp]),
        "gf_cube_batch_offsets": (i32, [vp, vp, vp, vp, vp]),
        "gf_cube_set_kernels": (i32, [vp, vp, vp, vp, i32]),
        "gf_cube_model": (i32, [vp, vp, vp, i32, i32, vp]),
        "gf_cube_chi2": (i32, [vp, vp, vp, i32, i32, vp, vp, vp]),
        "gf_cube_jacobian": (i32, [vp, vp, vp, i32, i32, vp]),
        "gf_cube_fit_lm": (i32, [vp, vp, vp, vp, vp, ctypes.POINTER(GfLmOpts), i32, vp]),
        "gf_version": (ctypes.c_char_p, []),
        "gf_tune_form_get": (i32, [vp, i32]),
        "gf_tune_form_set": (i32, [vp, i32, i32]),
        "gf_tune_min_active_get": (i32, [vp, i32]),
        "gf_tune_min_active_set": (i32, [vp, i32, i32]),
        "gf_tune_direct_get": (i32, [vp]),
        "gf_tune_direct_set": (i32, [vp, i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return _lib


def check(status: int, ctx=None, what: str = "") -> None:
    if status != GF_OK:
        msg = lib().gf_last_error(ctx).decode() if ctx else what
        raise GfError(status, msg or what)


# Thin wrappers with the C names (pointers as ints).
def gf_create(device: int = 0, autotune_cache=None) -> int:
    p = ctypes.c_void_p()
    path = None if autotune_cache is None else os.fsencode(autotune_cache)
    check(lib().gf_create(ctypes.byref(p), device, path), None, "gf_create failed")
    return p.value


def gf_chi2_noalloc(ctx, b, model_ptr, theta_ptr, data_ptr, weight_ptr, resid_ptr, chi2_ptr) -> None:
    check(lib().gf_chi2_noalloc(ctx, b, model_ptr, theta_ptr, data_ptr, weight_ptr, resid_ptr, chi2_ptr), ctx)


def gf_autotune(ctx, sides=None) -> None:
    import numpy as np
    if not sides:
        check(lib().gf_autotune(ctx, None, 0), ctx)
        return
    a = np.ascontiguousarray(sides, dtype=np.int32)
    check(lib().gf_autotune(ctx, a.ctypes.data, a.size), ctx)


def gf_destroy(ctx: int) -> None:
    lib().gf_destroy(ctx)


def gf_set_stream(ctx: int, stream: int) -> None:
    check(lib().gf_set_stream(ctx, stream), ctx)


def gf_synchronize(ctx: int) -> None:
    check(lib().gf_synchronize(ctx), ctx)


def gf_batch_create(ctx: int, H, W, K, ncomp, shared: bool) -> int:
    n = len(H)
    arr = ctypes.c_int32 * n
    h, w, k, c = arr(*H), arr(*W), arr(*K), arr(*ncomp)
    p = ctypes.c_void_p()
    check(lib().gf_batch_create(ctx, n, h, w, k, c, int(shared), ctypes.byref(p)), ctx)
    return p.value


def gf_batch_create_grouped(ctx: int, H, W, K, ncomp, group) -> int:
    n = len(H)
    arr = ctypes.c_int32 * n
    h, w, k, c, g = arr(*H), arr(*W), arr(*K), arr(*ncomp), arr(*group)
    p = ctypes.c_void_p()
    check(lib().gf_batch_create_grouped(ctx, n, h, w, k, c, g, ctypes.byref(p)), ctx)
    return p.value


def gf_batch_groups(b: int) -> int:
    return int(lib().gf_batch_groups(b))


def gf_group_best(ctx, b, res_ptr, theta_ptr, best_ptr, stamp_ptr):
    check(lib().gf_group_best(ctx, b, res_ptr, theta_ptr, best_ptr, stamp_ptr), ctx)


def gf_expand_starts(ctx, n_groups, n_starts, theta0_ptr, out_ptr):
    check(lib().gf_expand_starts(ctx, int(n_groups), int(n_starts), theta0_ptr, out_ptr), ctx)


def gf_batch_destroy(b: int) -> None:
    lib().gf_batch_destroy(b)


def gf_batch_sizes(b: int) -> dict:
    v = [ctypes.c_int64() for _ in range(6)]
    check(lib().gf_batch_sizes(b, *[ctypes.byref(x) for x in v]), None, "gf_batch_sizes failed")
    return dict(zip(("n_pix", "n_pad", "n_psf", "n_par", "n_img", "n_jac"), (x.value for x in v)))


def gf_batch_offsets(b: int, n: int) -> dict:
    arrs = [(ctypes.c_int64 * n)() for _ in range(6)]
    check(lib().gf_batch_offsets(b, *arrs), None, "gf_batch_offsets failed")
    return dict(zip(("pix", "pad", "psf", "par", "img", "jac"), ([int(v) for v in a] for a in arrs)))


def gf_psf_prepare(ctx: int, b: int, taps_ptr: int, mode: int) -> int:
    p = ctypes.c_void_p()
    check(lib().gf_psf_prepare(ctx, b, taps_ptr, mode, ctypes.byref(p)), ctx)
    return p.value


def gf_psf_destroy(p: int) -> None:
    lib().gf_psf_destroy(p)


def gf_psf_paths(p: int, n: int):
    f = (ctypes.c_int32 * n)()
    s = (ctypes.c_int32 * n)()
    check(lib().gf_psf_paths(p, f, s), None, "gf_psf_paths failed")
    return list(f), list(s)


def gf_eval_model(ctx, b, theta_ptr, oversample, out_ptr):
    check(lib().gf_eval_model(ctx, b, theta_ptr, oversample, out_ptr), ctx)


def gf_convolve_psf(ctx, b, psf, in_ptr, n_ch, out_ptr):
    check(lib().gf_convolve_psf(ctx, b, psf, in_ptr, n_ch, out_ptr), ctx)


def gf_model(ctx, b, psf, theta_ptr, oversample, out_ptr, work_ptr):
    check(lib().gf_model(ctx, b, psf, theta_ptr, oversample, out_ptr, work_ptr), ctx)


def gf_chi2(ctx, b, model_ptr, theta_ptr, data_ptr, weight_ptr, resid_ptr, chi2_ptr):
    check(lib().gf_chi2(ctx, b, model_ptr, theta_ptr, data_ptr, weight_ptr, resid_ptr, chi2_ptr), ctx)


def gf_likelihood(ctx, b, psf, theta_ptr, oversample, data_ptr, weight_ptr, chi2_ptr, work_ptr):
    check(lib().gf_likelihood(ctx, b, psf, theta_ptr, oversample, data_ptr, weight_ptr, chi2_ptr, work_ptr), ctx)


def gf_likelihood_workspace(b, psf) -> int:
    return int(lib().gf_likelihood_workspace(b, psf))


def gf_jacobian(ctx, b, psf, theta_ptr, oversample, mode, cot_ptr, weight_ptr, scale, out_ptr):
    check(lib().gf_jacobian(ctx, b, psf, theta_ptr, oversample, mode, cot_ptr, weight_ptr, float(scale), out_ptr),
          ctx)


def gf_lm_opts_default() -> GfLmOpts:
    o = GfLmOpts()
    lib().gf_lm_opts_default(ctypes.byref(o))
    return o


def gf_fit_lm(ctx, b, psf, data_ptr, weight_ptr, theta_ptr, opts: GfLmOpts, res_ptr):
    check(lib().gf_fit_lm(ctx, b, psf, data_ptr, weight_ptr, theta_ptr, ctypes.byref(opts), res_ptr), ctx)


def gf_line_batch_create(ctx: int, N, K, n_lines) -> int:
    import numpy as np
    n = len(N)
    a = [np.ascontiguousarray(v, dtype=np.int32) for v in (N, K, n_lines)]
    out = ctypes.c_void_p()
    check(lib().gf_line_batch_create(ctx, n, *[x.ctypes.data for x in a], ctypes.byref(out)), ctx)
    return out.value


def gf_line_batch_destroy(lb: int) -> None:
    lib().gf_line_batch_destroy(lb)


def gf_line_batch_offsets(lb: int, n: int) -> dict:
    import numpy as np
    arrs = {k: np.zeros(n + 1, np.int64) for k in ("data", "lsf", "par")}
    check(lib().gf_line_batch_offsets(lb, *[arrs[k].ctypes.data for k in ("data", "lsf", "par")]))
    return arrs


def gf_line_model(ctx, lb, lsf_ptr, theta_ptr, oversample, out_ptr):
    check(lib().gf_line_model(ctx, lb, lsf_ptr, theta_ptr, oversample, out_ptr), ctx)


def gf_line_chi2(ctx, lb, lsf_ptr, theta_ptr, oversample, data_ptr, weight_ptr, chi2_ptr):
    check(lib().gf_line_chi2(ctx, lb, lsf_ptr, theta_ptr, oversample, data_ptr, weight_ptr, chi2_ptr), ctx)


def gf_line_fit_lm(ctx, lb, lsf_ptr, data_ptr, weight_ptr, theta_ptr, opts: GfLmOpts, res_ptr):
    check(lib().gf_line_fit_lm(ctx, lb, lsf_ptr, data_ptr, weight_ptr, theta_ptr, ctypes.byref(opts), res_ptr), ctx)


def gf_cube_batch_create(ctx: int, H, W, K, n_chan: int, k_lsf: int) -> int:
    import numpy as np
    n = len(H)
    a = [np.ascontiguousarray(v, dtype=np.int32) for v in (H, W, K)]
    out = ctypes.c_void_p()
    check(lib().gf_cube_batch_create(ctx, n, *[x.ctypes.data for x in a], int(n_chan), int(k_lsf),
                                     ctypes.byref(out)), ctx)
    return out.value


def gf_cube_batch_destroy(cb: int) -> None:
    lib().gf_cube_batch_destroy(cb)


def gf_cube_batch_offsets(cb: int, n: int) -> dict:
    import numpy as np
    keys = ("vox", "psf", "lsf", "par")
    arrs = {k: np.zeros(n + 1, np.int64) for k in keys}
    check(lib().gf_cube_batch_offsets(cb, *[arrs[k].ctypes.data for k in keys]))
    return arrs


def gf_cube_set_kernels(ctx, cb, psf_ptr, lsf_ptr, mode):
    check(lib().gf_cube_set_kernels(ctx, cb, psf_ptr, lsf_ptr, mode), ctx)


def gf_cube_model(ctx, cb, theta_ptr, oversample, oversample_v, out_ptr):
    check(lib().gf_cube_model(ctx, cb, theta_ptr, oversample, oversample_v, out_ptr), ctx)


def gf_cube_chi2(ctx, cb, theta_ptr, oversample, oversample_v, data_ptr, weight_ptr, chi2_ptr):
    check(lib().gf_cube_chi2(ctx, cb, theta_ptr, oversample, oversample_v, data_ptr, weight_ptr, chi2_ptr), ctx)


def gf_cube_jacobian(ctx, cb, theta_ptr, oversample, oversample_v, out_ptr):
    check(lib().gf_cube_jacobian(ctx, cb, theta_ptr, oversample, oversample_v, out_ptr), ctx)


def gf_cube_fit_lm(ctx, cb, data_ptr, weight_ptr, theta_ptr, opts: GfLmOpts, oversample_v, res_ptr):
    check(lib().gf_cube_fit_lm(ctx, cb, data_ptr, weight_ptr, theta_ptr, ctypes.byref(opts), oversample_v, res_ptr),
          ctx)


def gf_profile_start(ctx):
    check(lib().gf_profile_start(ctx), ctx)


def gf_profile_stop(ctx):
    check(lib().gf_profile_stop(ctx), ctx)


def gf_profile_read(ctx) -> dict:
    """{kernel name: (launches, total ms)} of the timed launches."""
    n = lib().gf_profile_kernels(ctx)
    if n < 0:
        raise GfError(GF_EDEVICE, "gf_profile_kernels failed")
    out = {}
    for i in range(n):
        buf = ctypes.create_string_buffer(128)
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        check(lib().gf_profile_get(ctx, i, buf, 128, ctypes.byref(cnt), ctypes.byref(ms)), ctx)
        out[buf.value.decode()] = (int(cnt.value), float(ms.value))
    return out


def gf_tune_form_get(ctx, L: int) -> int:
    return int(lib().gf_tune_form_get(ctx, L))


def gf_tune_form_set(ctx, L: int, form: int) -> None:
    check(lib().gf_tune_form_set(ctx, L, form), ctx)


def gf_tune_min_active_get(ctx, L: int) -> int:
    return int(lib().gf_tune_min_active_get(ctx, L))


def gf_tune_min_active_set(ctx, L: int, n: int) -> None:
    check(lib().gf_tune_min_active_set(ctx, L, n), ctx)


def gf_tune_direct_get(ctx) -> int:
    return int(lib().gf_tune_direct_get(ctx))


def gf_tune_direct_set(ctx, k: int) -> None:
    check(lib().gf_tune_direct_set(ctx, int(k)), ctx)


def gf_version() -> str:
    return lib().gf_version().decode()


# ---------------------------------------------------------------- starting points
def gf_moments_guess(ctx, b, data_ptr, theta_ptr):
    check(lib().gf_moments_guess(ctx, b, data_ptr, theta_ptr), ctx)


def gf_cnn_create(ctx: int, side: int, max_batch: int) -> int:
    p = ctypes.c_void_p()
    check(lib().gf_cnn_create(ctx, side, max_batch, ctypes.byref(p)), ctx)
    return p.value


def gf_cnn_destroy(cnn: int) -> None:
    lib().gf_cnn_destroy(cnn)


def gf_cnn_param_count(cnn: int) -> int:
    return int(lib().gf_cnn_param_count(cnn))


def gf_cnn_init(ctx, cnn, key: int):
    check(lib().gf_cnn_init(cnn, key), ctx)


def gf_cnn_set_params(ctx, cnn, params_ptr):
    check(lib().gf_cnn_set_params(cnn, params_ptr), ctx)


def gf_cnn_get_params(ctx, cnn, out_ptr):
    check(lib().gf_cnn_get_params(cnn, out_ptr), ctx)


def gf_cnn_forward(ctx, cnn, stamps_ptr, n, out_ptr):
    check(lib().gf_cnn_forward(cnn, stamps_ptr, n, out_ptr), ctx)


def gf_cnn_gradients(ctx, cnn, stamps_ptr, targets_ptr, n, grads_ptr, loss_ptr):
    check(lib().gf_cnn_gradients(cnn, stamps_ptr, targets_ptr, n, grads_ptr, loss_ptr), ctx)


def gf_cnn_train_step(ctx, cnn, stamps_ptr, targets_ptr, n, lr, loss_ptr):
    check(lib().gf_cnn_train_step(cnn, stamps_ptr, targets_ptr, n, float(lr), loss_ptr), ctx)


def gf_cnn_steps(cnn) -> int:
    return int(lib().gf_cnn_steps(cnn))


def gf_cnn_encode(ctx, n, side, theta_ptr, targets_ptr):
    check(lib().gf_cnn_encode(ctx, n, side, theta_ptr, targets_ptr), ctx)


def gf_cnn_decode(ctx, n, side, targets_ptr, theta_ptr):
    check(lib().gf_cnn_decode(ctx, n, side, targets_ptr, theta_ptr), ctx)


def _counter(ctr):
    c = (ctypes.c_uint64 * 4)(*[int(v) & ((1 << 64) - 1) for v in (list(ctr) + [0, 0, 0, 0])[:4]])
    return c


def gf_philox(ctx, key0, key1, ctr, n_blocks, out_ptr):
    check(lib().gf_philox(ctx, key0, key1, _counter(ctr), n_blocks, out_ptr), ctx)


def gf_normal_noise(ctx, n, sigma, key0, key1, ctr, clean_ptr, out_ptr):
    check(lib().gf_normal_noise(ctx, n, float(sigma), key0, key1, _counter(ctr), clean_ptr, out_ptr), ctx)


def gf_draw_prior(ctx, n, side, key0, key1, ctr, theta_ptr):
    check(lib().gf_draw_prior(ctx, n, side, key0, key1, _counter(ctr), theta_ptr), ctx)


def gf_probe(ctx, kind: int, n: int, reps: int) -> float:
    r = ctypes.c_double()
    check(lib().gf_probe(ctx, int(kind), int(n), int(reps), ctypes.byref(r)), ctx)
    return r.value


# ---------------------------------------------------------------- MCMC
def gf_mcmc_opts_default() -> GfMcmcOpts:
    o = GfMcmcOpts()
    lib().gf_mcmc_opts_default(ctypes.byref(o))
    return o


def gf_mcmc_run(ctx, b, psf, data_ptr, weight_ptr, theta_ptr, chi2_ptr, opts: GfMcmcOpts, samples_ptr, acc_ptr):
    check(lib().gf_mcmc_run(ctx, b, psf, data_ptr, weight_ptr, theta_ptr, chi2_ptr, ctypes.byref(opts), samples_ptr,
                            acc_ptr), ctx)


# ---------------------------------------------------------------- simplex
def gf_simplex_opts_default() -> GfSimplexOpts:
    o = GfSimplexOpts()
    lib().gf_simplex_opts_default(ctypes.byref(o))
    return o


def gf_fit_simplex(ctx, b, psf, data_ptr, weight_ptr, theta_ptr, opts: GfSimplexOpts, res_ptr, trace_ptr, trace_cap):
    check(lib().gf_fit_simplex(ctx, b, psf, data_ptr, weight_ptr, theta_ptr, ctypes.byref(opts), res_ptr, trace_ptr,
                               int(trace_cap)), ctx)
