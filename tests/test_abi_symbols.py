"""The C-ABI library loads and exports every entry point include/tsgmres.h
declares (no GPU needed: nothing is called)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsgmres.h")
LIB = os.path.join(ROOT, "paper_2608_11091_amd", "libtsgmres.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_five_calls():
    names = _declared()
    for n in ("tucker_apply_op", "tucker_rhosvd", "tucker_sketch", "tsgmres_solve", "tsgmres_backward"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n
    from paper_2608_11091_amd import _abi
    assert sorted(_abi.EXPORTS) == _declared()
    assert _abi.load().tk_version() == _abi.ABI_VERSION


def test_storage_helper_matches_worked_example():
    # Deblurring right-hand side of Sec. 4.3 (fixture tests/golden/storage_example.json)
    import json
    import os
    from paper_2608_11091_amd.api import storage_floats
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "storage_example.json")))
    assert storage_floats(g["n"], g["ranks"]) == g["tucker_floats"]
