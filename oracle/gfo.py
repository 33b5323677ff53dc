"""ctypes binding of the FP64 CPU oracle (``oracle/gfo.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this module to check the GPU library.  It imports
nothing from the GPU package and the GPU package never imports it.

Every function takes and returns float64 numpy arrays.  Parameter vectors are
``[x0, y0, Ie, Re, n, q, phi] * ncomp + [sky]`` (phi in radians), so
``ncomp = (len(theta) - 1) // 7``.  Which passage of Barsdell, Barnes & Fluke
(Sec. 2, steps 1-5; Sec. 3, transform / FFT / reduce) each function follows is
stated in the C source next to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gfo.c")
_LIB_PATH = os.path.join(_HERE, "libgfo.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile ``gfo.c`` into ``libgfo.so`` next to it (gcc, FP64, OpenMP).

    ``-ffp-contract=off`` keeps every product and sum rounded as written.
    """
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-march=x86-64-v2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def use_native(build_dir: str) -> str:
    """Rebuild the oracle for the host it runs on (``-O3 -march=native``, the
    same ``-ffp-contract=off`` rounding, hence the same results) into
    ``build_dir`` and load that copy instead.  Used by the CPU-baseline leg of
    the benchmark only: the tests keep the portable build."""
    global _lib
    os.makedirs(build_dir, exist_ok=True)
    path = os.path.join(build_dir, "libgfo_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", path,
           "-lm"]
    subprocess.run(cmd, check=True)
    _lib = None
    _load(path)
    return path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _load(_LIB_PATH)
    return _lib


def _load(path):
    global _lib
    if _lib is None:
        L = ctypes.CDLL(path)
        i, d, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.gfo_gammp.restype = d
        L.gfo_gammp.argtypes = [d, d]
        L.gfo_dgammp_dx.restype = d
        L.gfo_dgammp_dx.argtypes = [d, d]
        L.gfo_bn.restype = d
        L.gfo_bn.argtypes = [d]
        L.gfo_dbn.restype = d
        L.gfo_dbn.argtypes = [d]
        L.gfo_sersic_point.restype = d
        L.gfo_sersic_point.argtypes = [vp, d, d]
        L.gfo_pixel.restype = d
        L.gfo_pixel.argtypes = [i, vp, i, i, i]
        L.gfo_eval_padded.restype = None
        L.gfo_eval_padded.argtypes = [i, i, i, i, vp, i, vp]
        L.gfo_eval_padded_comps.restype = None
        L.gfo_eval_padded_comps.argtypes = [i, i, i, i, vp, i, vp]
        L.gfo_conv_valid.restype = None
        L.gfo_conv_valid.argtypes = [vp, i, i, vp, i, vp]
        L.gfo_conv_valid_pixel.restype = d
        L.gfo_conv_valid_pixel.argtypes = [vp, i, i, vp, i, i, i]
        L.gfo_model.restype = None
        L.gfo_model.argtypes = [i, i, i, i, vp, i, vp, vp]
        L.gfo_chi2.restype = d
        L.gfo_chi2.argtypes = [ctypes.c_long, vp, vp, vp, vp]
        L.gfo_dpixel.restype = None
        L.gfo_dpixel.argtypes = [i, vp, i, i, i, vp]
        L.gfo_dpadded.restype = None
        L.gfo_dpadded.argtypes = [i, i, i, i, vp, i, vp]
        L.gfo_jacobian.restype = None
        L.gfo_jacobian.argtypes = [i, i, i, i, vp, i, vp, vp]
        L.gfo_grad_chi2.restype = None
        L.gfo_grad_chi2.argtypes = [i, i, i, i, vp, i, vp, vp, vp, vp]
        L.gfo_fit_lm.restype = i
        L.gfo_fit_lm.argtypes = [i, i, i, i, i, vp, vp, vp, vp, vp, vp, i, vp, vp, vp]
        L.gfo_set_threads.restype = None
        L.gfo_set_threads.argtypes = [i]
        L.gfo_get_threads.restype = i
        L.gfo_get_threads.argtypes = []
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ncomp(theta: np.ndarray) -> int:
    P = theta.shape[-1]
    if P < 8 or (P - 1) % 7:
        raise ValueError(f"parameter vector of length {P} is not 7*ncomp+1")
    return (P - 1) // 7


def set_threads(n: int) -> None:
    lib().gfo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().gfo_get_threads())


def gammp(a: float, x: float) -> float:
    return float(lib().gfo_gammp(a, x))


def bn(n: float) -> float:
    return float(lib().gfo_bn(n))


def dbn(n: float) -> float:
    return float(lib().gfo_dbn(n))


def sersic_point(comp7, x: float, y: float) -> float:
    c = _f64(comp7)
    return float(lib().gfo_sersic_point(_ptr(c), x, y))


def pixel(theta, S: int, i: int, j: int) -> float:
    """Pixel value (no sky) at stamp pixel (row i, col j); padding allowed."""
    t = _f64(theta)
    return float(lib().gfo_pixel(_ncomp(t), _ptr(t), S, i, j))


def eval_padded(H: int, W: int, K: int, theta, S: int = 5) -> np.ndarray:
    """Step 1 on the padded (H+K-1) x (W+K-1) grid, all components, no sky."""
    t = _f64(theta)
    out = np.empty((H + K - 1, W + K - 1), np.float64)
    lib().gfo_eval_padded(H, W, K, _ncomp(t), _ptr(t), S, _ptr(out))
    return out


def eval_padded_comps(H: int, W: int, K: int, theta, S: int = 5) -> np.ndarray:
    t = _f64(theta)
    nc = _ncomp(t)
    out = np.empty((nc, H + K - 1, W + K - 1), np.float64)
    lib().gfo_eval_padded_comps(H, W, K, nc, _ptr(t), S, _ptr(out))
    return out


def conv_valid(mp, psf) -> np.ndarray:
    """Step 2 as its definition: valid linear convolution of the padded grid."""
    mp = _f64(mp)
    psf = _f64(psf)
    K = psf.shape[0]
    Mh, Mw = mp.shape
    out = np.empty((Mh - K + 1, Mw - K + 1), np.float64)
    lib().gfo_conv_valid(_ptr(mp), Mh, Mw, _ptr(psf), K, _ptr(out))
    return out


def conv_valid_pixel(mp, psf, y: int, x: int) -> float:
    mp = _f64(mp)
    psf = _f64(psf)
    return float(lib().gfo_conv_valid_pixel(_ptr(mp), mp.shape[0], mp.shape[1], _ptr(psf), psf.shape[0], y, x))


def model(H: int, W: int, theta, psf, S: int = 5) -> np.ndarray:
    """Convolved model plus sky on the H x W stamp."""
    t = _f64(theta)
    psf = _f64(psf)
    out = np.empty((H, W), np.float64)
    lib().gfo_model(H, W, psf.shape[0], _ncomp(t), _ptr(t), S, _ptr(psf), _ptr(out))
    return out


def chi2(d, w, m, want_resid: bool = False):
    """Step 3: chi^2 = sum w (d - m)^2 (and resid = sqrt(w) (d - m))."""
    d, w, m = _f64(d), _f64(w), _f64(m)
    r = np.empty_like(d) if want_resid else None
    v = float(lib().gfo_chi2(d.size, _ptr(d), _ptr(w), _ptr(m), _ptr(r) if r is not None else None))
    return (v, r) if want_resid else v


def dpixel(theta, S: int, i: int, j: int) -> np.ndarray:
    t = _f64(theta)
    nc = _ncomp(t)
    out = np.empty(7 * nc, np.float64)
    lib().gfo_dpixel(nc, _ptr(t), S, i, j, _ptr(out))
    return out


def dpadded(H: int, W: int, K: int, theta, S: int = 5) -> np.ndarray:
    t = _f64(theta)
    nc = _ncomp(t)
    out = np.empty((7 * nc, H + K - 1, W + K - 1), np.float64)
    lib().gfo_dpadded(H, W, K, nc, _ptr(t), S, _ptr(out))
    return out


def jacobian(H: int, W: int, theta, psf, S: int = 5) -> np.ndarray:
    """d m / d theta images, shape [P, H, W] (last plane = d/d sky = 1)."""
    t = _f64(theta)
    psf = _f64(psf)
    out = np.empty((t.size, H, W), np.float64)
    lib().gfo_jacobian(H, W, psf.shape[0], _ncomp(t), _ptr(t), S, _ptr(psf), _ptr(out))
    return out


def grad_chi2(theta, psf, d, w, S: int = 5) -> np.ndarray:
    t = _f64(theta)
    psf, d, w = _f64(psf), _f64(d), _f64(w)
    H, W = d.shape
    out = np.empty(t.size, np.float64)
    lib().gfo_grad_chi2(H, W, psf.shape[0], _ncomp(t), _ptr(t), S, _ptr(psf), _ptr(d), _ptr(w), _ptr(out))
    return out


LM_DEFAULTS = dict(max_iter=100, lambda0=1e-3, lambda_up=10.0, lambda_down=10.0, lambda_max=1e10,
                   ftol=1e-5, xtol=1e-10)


def fit_lm(theta0, psf, d, w, S: int = 5, free=None, lo=None, hi=None, **opts):
    """Levenberg-Marquardt fit (steps 4-5).  Returns (theta, info dict)."""
    o = dict(LM_DEFAULTS)
    o.update(opts)
    t = _f64(theta0).copy()
    psf, d, w = _f64(psf), _f64(d), _f64(w)
    H, W = d.shape
    P = t.size
    fm = None if free is None else np.ascontiguousarray(free, dtype=np.uint8)
    lo_ = None if lo is None else _f64(lo)
    hi_ = None if hi is None else _f64(hi)
    dopt = np.array([o["lambda0"], o["lambda_up"], o["lambda_down"], o["lambda_max"], o["ftol"], o["xtol"]],
                    np.float64)
    rd = np.zeros(2, np.float64)
    ri = np.zeros(5, np.int32)
    if P > 64:
        raise ValueError("at most 64 parameters")
    rc = lib().gfo_fit_lm(H, W, psf.shape[0], _ncomp(t), S, _ptr(psf), _ptr(d), _ptr(w),
                          _ptr(fm) if fm is not None else None,
                          _ptr(lo_) if lo_ is not None else None,
                          _ptr(hi_) if hi_ is not None else None,
                          int(o["max_iter"]), _ptr(dopt), _ptr(t), _ptr(rd), _ptr(ri))
    if rc != 0:
        raise ValueError("invalid arguments to the oracle LM")
    info = dict(chi2=float(rd[0]), lam=float(rd[1]), iters=int(ri[0]), nfev=int(ri[1]), njev=int(ri[2]),
                status=int(ri[3]), reason=int(ri[4]))
    return t, info
