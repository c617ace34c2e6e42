"""The C-ABI library loads and exports every function the public headers
declare (no GPU needed: nothing is called)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1902_01061_amd", "libsgreg.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"^\s*(?:int|const char\*|void)\s+(sgr_\w+)\s*\(", txt, flags=re.M))
    return sorted(names)


def test_headers_declare_the_api():
    names = _declared()
    for must in ("sgr_create", "sgr_destroy", "sgr_last_error", "sgr_descriptors", "sgr_step", "sgr_register",
                 "sgr_residual"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libsgreg.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_header_structs():
    from paper_1902_01061_amd import _ffi
    assert ctypes.sizeof(_ffi.SgrCloud) == 40
    assert ctypes.sizeof(_ffi.SgrParams) == 56
    for n in _ffi.SIGNATURES:
        assert n in _declared()
