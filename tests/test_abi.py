"""The C-ABI library loads and exports every entry point include/bm.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2512_14193_amd import binding, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "bm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(bm_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        build.build(verbose=False)
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTED) == names


def test_strerror_without_device():
    lib = binding.lib()
    assert lib.bm_strerror(0) == b"ok"
    assert lib.bm_strerror(-1) == b"invalid argument"
    assert b"singular" in lib.bm_strerror(3)
