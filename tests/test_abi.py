"""The C ABI: the library loads and exports every function include/dd.h declares
(no device calls), and the binding's signatures cover exactly that set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dd.h")
LIB = os.path.join(ROOT, "paper_1811_00355_amd", "libdd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dd_\w+)\s*\(", text)
    return sorted(set(names))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared in dd.h but not exported: {missing}"


def test_binding_covers_the_header():
    from paper_1811_00355_amd import binding
    assert sorted(binding.SIGNATURES) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_status_strings_without_a_device():
    lib = ctypes.CDLL(LIB)
    lib.dd_status_str.restype = ctypes.c_char_p
    assert lib.dd_status_str(0) == b"DD_OK"
    assert lib.dd_status_str(4) == b"DD_EBUDGET"
    assert lib.dd_status_str(99) == b"DD_UNKNOWN"
