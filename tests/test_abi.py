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
        pytest.fail("libsgreg.so is not built (run build.py)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_header_structs(tmp_path):
    """Every field offset and the size of the header's structs, as a C
    compiler lays them out, against the ctypes mirrors."""
    import shutil
    import subprocess

    from paper_1902_01061_amd import _ffi
    for n in _ffi.SIGNATURES:
        assert n in _declared()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"sgr_cloud": _ffi.SgrCloud, "sgr_params": _ffi.SgrParams, "sgr_level": _ffi.SgrLevel}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "sgreg.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
