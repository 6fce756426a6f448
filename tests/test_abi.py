"""The C-ABI library builds, loads and exports every function declared in
include/lbfd.h (no compute call: runs on CPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbfd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbfd_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lbfd_init", "lbfd_step", "lbfd_read_fields", "lbfd_diagnostics", "lbfd_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2304_05657_amd import build, lbfd
    if not os.path.exists(lbfd.LIB_PATH):
        build.build()
    lib = ctypes.CDLL(lbfd.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(lbfd.EXPORTS) == set(declared_functions())


def test_error_strings_without_device():
    from paper_2304_05657_amd import lbfd
    lib = lbfd.load_library()
    assert lib.lbfd_strerror(0) == b"ok"
    assert lib.lbfd_strerror(-4) == b"non-finite state"
    assert lib.lbfd_level(None) == -1
