"""The C-ABI library loads and exports every entry point that include/nsmf.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nsmf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nsmf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_api():
    names = declared_functions()
    for need in ["nsmf_upload_mesh", "nsmf_set_state", "nsmf_residual", "nsmf_jacobian_apply", "nsmf_residual_vjp"]:
        assert need in names


def test_library_exports_all_declared_symbols():
    from paper_1406_6573_amd.nsmf import LIB_PATH, EXPORTED
    if not os.path.exists(LIB_PATH):
        pytest.fail("libnsmf.so not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(EXPORTED) == declared_functions()
    lib.nsmf_version.restype = ctypes.c_char_p
    assert lib.nsmf_version().startswith(b"nsmf")


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1406_6573_amd import nsmf
    with pytest.raises(RuntimeError):
        nsmf._lib_saved = nsmf._lib
        nsmf._lib = None
        try:
            nsmf.load_library(str(tmp_path / "missing.so"))
        finally:
            nsmf._lib = nsmf._lib_saved
