"""CPU-side checks of the C ABI library: it loads, exports every declared symbol, and
rejects bad arguments before touching a device (no compute on the CPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qaoa.h")).read()
    return sorted(set(re.findall(r"\b(qaoa_[a-z_]+)\s*\(", src)))


def test_header_declarations_are_exported():
    import paper_2312_06451_amd._lib as L
    lib = L.lib()
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTED) == names


def test_status_strings_and_null_args():
    import ctypes
    import paper_2312_06451_amd._lib as L
    lib = L.lib()
    assert lib.qaoa_status_string(0) == b"ok"
    assert lib.qaoa_status_string(-4) == b"unsupported"
    assert lib.qaoa_ctx_create(0, None) == L.QAOA_ERR_INVALID_ARG
    assert b"NULL" in lib.qaoa_last_error()
    assert lib.qaoa_ctx_destroy(None) == 0
    assert lib.qaoa_problem_destroy(None) == 0
    assert lib.qaoa_mixer_destroy(None) == 0
    assert lib.qaoa_expect(None, None, 1, None, None, 0, None, None) == L.QAOA_ERR_INVALID_ARG
    out = ctypes.c_void_p()
    assert lib.qaoa_mixer_x(None, 4, ctypes.byref(out)) == L.QAOA_ERR_INVALID_ARG


def test_no_oracle_on_product_path():
    # the library and its Python package never reference the test oracle
    pkg = os.path.join(ROOT, "paper_2312_06451_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text, f
