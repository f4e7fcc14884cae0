"""The C-ABI library loads and exports every function that include/celeste.h declares.
No compute calls: this runs without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "celeste.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(celeste_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["celeste_plan_create", "celeste_plan_destroy", "celeste_elbo", "celeste_elbo_grad",
              "celeste_hvp", "celeste_sweep", "celeste_newton", "celeste_status_string", "celeste_version"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1801_10277_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libceleste.so not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert set(declared()) == set(binding.EXPORTS)
    lib.celeste_version.restype = ctypes.c_int
    assert lib.celeste_version() == 7
    lib.celeste_status_string.restype = ctypes.c_char_p
    assert lib.celeste_status_string(-2) == b"batch members share pixels"
