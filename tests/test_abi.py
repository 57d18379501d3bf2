"""The C ABI library: it loads without a GPU and exports every declared entry point."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "matprobe.h")
LIB = os.path.join(ROOT, "paper_1101_3615_amd", "libmatprobe.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mp_[a-zA-Z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build first: python -m paper_1101_3615_amd.build"
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_error_strings_without_device():
    lib = ctypes.CDLL(LIB)
    lib.mp_strerror.restype = ctypes.c_char_p
    assert lib.mp_strerror(0) == b"ok"
    assert lib.mp_strerror(-2).startswith(b"out of device memory")
    assert lib.mp_strerror(-99) == b"unknown error"
    # argument validation happens before any device call
    lib.mp_last_error.restype = ctypes.c_char_p
    assert lib.mp_create(None, None, None, None) == -1
    assert b"null" in lib.mp_last_error()


def test_python_binding_imports_without_device():
    import paper_1101_3615_amd as M
    assert callable(M.probe_fit) and callable(M.apply_Hinv)
    from paper_1101_3615_amd._lib import EXPORTS
    assert set(EXPORTS) <= set(declared())
