"""CPU-side checks of the C ABI: the built library loads and exports every
function that include/oem.h declares; host-side argument checks."""
import ctypes
import os
import re

import pytest

import paper_1801_09661_amd as oem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "oem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(oem_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(oem.LIB_PATH):
        pytest.fail("liboem.so is not built; run __graft_entry__.build()")
    return oem.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["oem_gram_create", "oem_gram", "oem_fit_path", "oem_cv", "oem_gram_free",
                     "oem_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(oem.EXPORTED) <= set(_declared())


def test_version_string(lib):
    assert b"gfx950" in lib.oem_version()


def test_invalid_arguments_rejected_without_gpu(lib):
    h = ctypes.c_void_p()
    assert lib.oem_gram_create(0, 1, 0, 0, 0, ctypes.byref(h)) == oem.OEM_E_INVAL
    assert b"p must be" in lib.oem_last_error()
    assert lib.oem_gram_create(10, 0, 0, 0, 0, ctypes.byref(h)) == oem.OEM_E_INVAL
    assert lib.oem_gram_create(10, 2, 7, 0, 0, ctypes.byref(h)) == oem.OEM_E_INVAL
    assert lib.oem_gram_create(10, 2, 0, 9, 0, ctypes.byref(h)) == oem.OEM_E_INVAL
    assert lib.oem_gram(None, None, 0, 0, None, 0, None, None) == oem.OEM_E_INVAL
    assert lib.oem_fit_path(None, -1, None, 0, None, None, None, None, None, None, None,
                            None) == oem.OEM_E_INVAL
    assert lib.oem_cv(None, None, 0, None, None, None, None, None, None, None, None, None, None,
                      None) == oem.OEM_E_INVAL
    b = ctypes.c_void_p()
    pen = (oem.oem_penalty * 1)(oem.oem_penalty(oem.OEM_LASSO, 0.0, 0.0, 0.0))
    opts = oem.oem_path_opts(10, 1e-3, None, 1e-10, 100, 1, None, None, None, 0)
    assert lib.oem_batch_create(None, 0, 0, 0, pen, 1, ctypes.byref(opts), ctypes.byref(b)) == oem.OEM_E_INVAL
    recs = (oem.oem_problem * 1)(oem.oem_problem(0, 10, 10, None, None, None, None, None, None, None))
    assert lib.oem_batch_create(recs, 1, 0, 0, pen, 1, ctypes.byref(opts), ctypes.byref(b)) == oem.OEM_E_INVAL
    assert b"bad p" in lib.oem_last_error()
    opts.standardize = 0
    assert lib.oem_batch_create(recs, 1, 0, 0, pen, 1, ctypes.byref(opts), ctypes.byref(b)) == oem.OEM_E_INVAL
    assert lib.oem_batch_run(None, None) == oem.OEM_E_INVAL
    assert lib.oem_gram_autotune(None, None, 0, 0, None, None) == oem.OEM_E_INVAL


def test_no_cpu_fallback_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(oem.OemError):
        oem.oem_gram_create(10)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 7, 100, 129])
def test_gram_loader_columns_stay_in_row(lib, p):
    """The Gram loaders' column choice (shared with the kernels) never reads
    past column p - 1 of a row, for every 4-column group of the padded
    panels, with and without 16-byte loads; so the last row's reads end
    inside X: largest index < (n - 1) ldx + p."""
    f = lib.oem_debug_gram_load_columns
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    cols = (ctypes.c_int32 * 4)()
    for vec_ok in (0, 1):
        for col in range(0, ((p + 127) // 128) * 128 + 128, 4):
            rc = f(p, col, vec_ok, cols)
            assert rc in (0, 1)
            assert all(0 <= c < p for c in cols), (p, col, vec_ok, list(cols))
            if col + 3 < p:
                assert list(cols) == [col, col + 1, col + 2, col + 3]
