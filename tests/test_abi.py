"""The C-ABI library loads and exports every entry point include/mr1l.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mr1l.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^(?:mr1l_status|const char\*|int)\s+(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_core_entry_points():
    names = _declared()
    for n in ("mr1l_plan", "mr1l_forward", "mr1l_adjoint", "mr1l_construct", "sfft_detect", "mr1l_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1711_05152_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmr1l.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.EXPORTED) <= set(_declared())


def test_binding_loads_and_reports_version():
    from paper_1711_05152_amd import _lib
    assert b"mr1l" in _lib.lib().mr1l_version()
    assert _lib.lib().mr1l_last_error() == b""


def test_build_flags_disable_packed_fp32():
    from paper_1711_05152_amd import build
    flags = " ".join(build.FLAGS)
    assert "-packed-fp32-ops" in flags and "--offload-arch=gfx950" in flags


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_1711_05152_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


def test_struct_layouts_match_the_binding(tmp_path):
    """sizeof and field offsets of the C-ABI structs (compiled from include/mr1l.h by the host C
    compiler) equal those of the ctypes structures the binding passes."""
    import shutil
    import subprocess
    from paper_1711_05152_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"sfft_params": _lib.SfftParams, "sfft_stats": _lib.SfftStats, "sfft_planted": _lib.SfftPlanted,
               "sfft_bspline": _lib.SfftBspline}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mr1l.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)
