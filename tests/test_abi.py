"""Host-side checks of the C ABI library (no GPU work is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(gf_[a-z_0-9]+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("gf_eval_model", "gf_convolve_psf", "gf_chi2", "gf_jacobian", "gf_fit_lm"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1101_2254_amd import _lib
    L = _lib.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(_lib.EXPORTS)
    assert "gfx950" in _lib.gf_version()


def test_lm_struct_layout_matches_header():
    from paper_1101_2254_amd import _lib
    o = _lib.gf_lm_opts_default()
    assert o.max_iter == 100 and o.oversample == 5 and o.lambda0 == 1e-3 and o.lambda_max == 1e10
    assert o.ftol == 1e-5 and o.poll_every == 4 and o.use_graph == 1 and o.speculate == -1 and o.start is None
    # the library's sizeof(gf_lm_opts), which every call checks, is the
    # binding's layout
    assert o.struct_size == ctypes.sizeof(_lib.GfLmOpts) == 112
    assert ctypes.sizeof(_lib.GfLmResult) == 40
    from paper_1101_2254_amd.ops import LM_RESULT_DTYPE
    assert LM_RESULT_DTYPE.itemsize == 40


def test_null_arguments_are_rejected_without_a_device():
    from paper_1101_2254_amd import _lib
    L = _lib.lib()
    assert L.gf_eval_model(None, None, None, 5, None) == _lib.GF_EINVAL
    assert L.gf_fit_lm(None, None, None, None, None, None, None, None) == _lib.GF_EINVAL
    assert L.gf_batch_count(None) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1101_2254_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()
