"""Host-side checks of the C ABI: the library loads and exports every
function include/mhd.h declares; no GPU work is started."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mhd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z_]+)\s*\(", src)))


def test_header_declares_the_five_calls():
    names = _declared()
    for n in ("mhd_init", "mhd_rhs", "mhd_step", "mhd_step_adjoint", "mhd_reductions"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2405_02483_amd import lib
    path = lib.lib_path()
    if not os.path.exists(path):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    L = lib.load()          # dlopen works without a GPU; nothing is launched
    for n in _declared():
        assert hasattr(L, n)


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the public structs have the sizes and field offsets
    that a C compiler gives the header's structs."""
    import ctypes
    import shutil
    from paper_2405_02483_amd import lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    checks = []
    for cname, py in (("mhd_box", lib.MhdBox), ("mhd_params", lib.MhdParams),
                      ("mhd_stats", lib.MhdStats)):
        checks.append((cname, "", ctypes.sizeof(py)))
        for fname, _ in py._fields_:
            checks.append((cname, fname, getattr(py, fname).offset))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mhd.h"', "int main(void){"]
    for cname, fname, _ in checks:
        expr = "sizeof(%s)" % cname if not fname else "offsetof(%s, %s)" % (cname, fname)
        lines.append('printf("%%zu\\n", (size_t)%s);' % expr)
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [c[2] for c in checks]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built library every call path raises."""
    from paper_2405_02483_amd import lib
    monkeypatch.setattr(lib, "_LIB", None)
    monkeypatch.setenv("STAGGER_MHD_LIB", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="not built"):
        lib.load()
