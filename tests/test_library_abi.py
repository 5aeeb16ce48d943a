"""The C-ABI library loads and exports every function include/deblur.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "deblur.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(deblur_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["deblur_create", "deblur_apply_H", "deblur_apply_Ht", "deblur_solve_tiles", "deblur_consensus"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1705_06603_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(_lib.exported_symbols()) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1705_06603_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def _create_error(psfs, P=3, G=2):
    """deblur_create on PSFs that break the contract: the check comes before
    any HIP call, so this runs without a GPU."""
    from paper_1705_06603_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    import numpy as np
    L = _lib.lib()
    params = _lib.make_params(24, 2, 12, 2, G, P)
    psf = np.ascontiguousarray(psfs, dtype=np.float32)
    h = ctypes.c_void_p()
    rc = L.deblur_create(ctypes.byref(params), psf.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(h))
    assert not h.value
    return rc, L.deblur_last_error(None).decode()


def _unit_psfs(G=2, P=3):
    import numpy as np
    rng = np.random.default_rng(0)
    h = rng.random((G, G, P, P))
    return h / h.sum(axis=(2, 3), keepdims=True)


def test_create_rejects_a_negative_psf():
    psfs = _unit_psfs()
    psfs[1, 0, 0, 2] = -0.01
    psfs[1, 0, 1, 1] += 0.01                 # still sums to 1
    rc, msg = _create_error(psfs)
    assert rc == -1 and "negative" in msg and "node 2" in msg, msg


def test_create_rejects_a_psf_not_summing_to_one():
    psfs = _unit_psfs()
    psfs[0, 1] *= 2.0
    rc, msg = _create_error(psfs)
    assert rc == -1 and "sums to 2" in msg and "node 1" in msg, msg
    psfs = _unit_psfs()
    psfs[1, 1] *= 1.0 - 2e-4
    rc, msg = _create_error(psfs)
    assert rc == -1 and "node 3" in msg, msg


def test_create_rejects_a_smoothing_eps_whose_square_is_subnormal():
    """Smoothed TV needs eps^2 to be a normal float (eps >= 2^-63): the
    regulariser's reciprocal square root is then exact hardware rsq."""
    from paper_1705_06603_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    import numpy as np
    L = _lib.lib()
    psf = np.ascontiguousarray(_unit_psfs(), dtype=np.float32)
    for eps in (1e-20, 2.0 ** -64):
        params = _lib.make_params(24, 2, 12, 2, 2, 3, reg_param=eps)
        h = ctypes.c_void_p()
        rc = L.deblur_create(ctypes.byref(params), psf.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(h))
        assert rc == -1 and not h.value
        assert "2^-63" in L.deblur_last_error(None).decode()
