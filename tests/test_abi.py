"""The C-ABI library loads and exports every function include/oc.h declares
(no compute call, no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "oc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(oc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("oc_register_grid", "oc_register_cut_surface", "oc_cut", "oc_donor_search"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1711_07663_amd import oc
    lib = ctypes.CDLL(oc.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(oc.EXPORTS) == _declared()


def test_checked_library_exports_the_same_symbols():
    """The bounds-checked variant is the same ABI."""
    path = os.path.join(ROOT, "paper_1711_07663_amd", "liboc_checked.so")
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_refuses_missing_library(tmp_path):
    from paper_1711_07663_amd import oc
    import pytest
    saved = oc._lib
    oc._lib = None
    try:
        with pytest.raises(ImportError):
            oc.load(str(tmp_path / "missing.so"))
    finally:
        oc._lib = saved


def test_service_refuses_null_arguments_without_a_device():
    """The cut service checks its arguments before any HIP call."""
    from paper_1711_07663_amd import oc
    L = oc.load()
    t = ctypes.c_uint64(99)
    assert L.oc_submit(None, None, ctypes.byref(t)) == oc.OC_EINVAL
    assert L.oc_wait(None, 1, 0) == oc.OC_EINVAL
    assert L.oc_service_info(None, None) == oc.OC_EINVAL
    assert b"oc_service_info" in L.oc_last_error()
