"""The C-ABI libraries load and export every declared symbol (no compute, CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bse_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared("bse.h")
    for must in ["bse_create", "bse_set_packed", "bse_apply", "bse_solve", "bse_backward", "bse_strength",
                 "bse_destroy", "bse_status_string", "bse_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2504_10096_amd", "libbse.so")
    assert os.path.exists(path), "libbse.so is not built"
    lib = ctypes.CDLL(path)
    for name in _declared("bse.h"):
        assert hasattr(lib, name), name


def test_binding_lists_the_exports():
    import paper_2504_10096_amd as bse
    assert sorted(bse.EXPORTS) == _declared("bse.h")


def test_status_strings_without_gpu():
    import paper_2504_10096_amd as bse
    lib = bse.load_library()
    assert lib.bse_status_string(0) == b"ok"
    assert lib.bse_status_string(4) == b"M is not positive definite"
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    assert lib.bse_create(ctypes.byref(h), 0, 0, 0, None) == bse.ERR_INVALID_ARG
    assert lib.bse_create(None, 0, 10, 0, None) == bse.ERR_INVALID_ARG
    assert lib.bse_create(ctypes.byref(h), 7, 10, 0, None) == bse.ERR_INVALID_ARG


def test_product_does_not_reference_the_oracle():
    """The GPU path shares no code with the oracle and never imports it."""
    pkg = os.path.join(ROOT, "paper_2504_10096_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "bse_oracle" not in text and "liboracle" not in text, f


@pytest.mark.parametrize("lib", ["synth/libsynth.so", "synth/libsynth_dev.so", "oracle/liboracle.so"])
def test_aux_libraries_built(lib):
    assert os.path.exists(os.path.join(ROOT, lib))
