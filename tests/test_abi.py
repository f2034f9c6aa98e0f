"""The C-ABI library loads and exports every entry point declared in
include/fdemri.h (no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdemri.h")
LIB = os.path.join(ROOT, "paper_2307_12585_amd", "libfdemri.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdemri_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["fdemri_create", "fdemri_destroy", "fdemri_waveform", "fdemri_waveform_batch",
                     "fdemri_vjp", "fdemri_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfdemri.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfdemri.so not built")
def test_binding_lists_match_header():
    import paper_2307_12585_amd as fd
    assert sorted(fd.EXPORTED) == declared_functions()


def test_oracle_and_library_share_no_code():
    """The oracle never imports the HIP package and vice versa."""
    for dirpath, _, files in os.walk(os.path.join(ROOT, "oracle")):
        for fn in files:
            if fn.endswith(".py"):
                assert "paper_2307_12585_amd" not in open(os.path.join(dirpath, fn)).read()
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_2307_12585_amd")):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".inc")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt
