"""CPU checks of the C ABI library: it loads, exports every symbol mdx.h
declares, and the binding's structs have the C layout. No compute calls."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdx.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(mdx_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    import paper_2503_20541_amd as mdx
    names = _declared()
    assert len(names) >= 10
    lib = mdx.library()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(mdx.EXPORTED)


def test_error_strings():
    import paper_2503_20541_amd as mdx
    assert mdx.error_string(0) == "ok"
    for code in range(-8, 0):
        assert mdx.error_string(code) != "unknown error"
    assert mdx.error_string(-99) == "unknown error"


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layout_matches_header(tmp_path):
    import ctypes
    import paper_2503_20541_amd as mdx
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "mdx.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(mdx_system_desc),"
        " sizeof(mdx_info), offsetof(mdx_system_desc, ewald_delta),"
        " offsetof(mdx_system_desc, pme_grid), offsetof(mdx_info, alpha));"
        " printf(\"%zu %zu\\n\", offsetof(mdx_system_desc, options),"
        " offsetof(mdx_info, n_list_tiles)); return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [ctypes.sizeof(mdx.SystemDesc), ctypes.sizeof(mdx.Info), mdx.SystemDesc.ewald_delta.offset,
           mdx.SystemDesc.pme_grid.offset, mdx.Info.alpha.offset,
           mdx.SystemDesc.options.offset, mdx.Info.n_list_tiles.offset]
    assert [int(v) for v in out] == got


def test_binding_constants_match_header():
    import paper_2503_20541_amd as mdx
    text = open(HEADER).read()
    defs = re.findall(r"^#define\s+(MDX_\w+)\s+\(?(-?(?:0x[0-9a-fA-F]+|\d+))u?\)?", text, re.M)
    assert len(defs) >= 20
    for name, val in defs:
        assert hasattr(mdx, name), name
        assert getattr(mdx, name) == int(val, 0), name


def test_desc_marshalling_roundtrip():
    import numpy as np
    import paper_2503_20541_amd as mdx
    import synth
    s = synth.config_system("water375")
    d, keep = mdx.desc_from_system(s)
    assert d.n_atoms == s.n_atoms and d.n_exclusions == len(s.exclusions)
    assert d.n_bonds == len(s.bonds) and d.n_angles == len(s.angles)
    assert list(d.pme_grid) == list(s.pme_grid)
    assert d.charge[5] == pytest.approx(float(s.charge[5]))
    assert d.exclusions[1] == s.exclusions[0, 1]
    assert np.isclose(d.r_cut, float(s.r_cut))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs hipcc")
def test_fresh_checkout_builds_library_on_import(tmp_path):
    """A tree without libmdx.so (a fresh clone) builds it on first import."""
    pkg = "paper_2503_20541_amd"
    shutil.copytree(os.path.join(ROOT, pkg), tmp_path / pkg,
                    ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", ".libmdx.lock"))
    shutil.copytree(os.path.join(ROOT, "include"), tmp_path / "include")
    assert not (tmp_path / pkg / "libmdx.so").exists()
    code = ("import paper_2503_20541_amd as m; lib = m.library(); "
            "print(lib._name); [getattr(lib, n) for n in m.EXPORTED]")
    res = subprocess.run(["python", "-c", code], cwd=tmp_path, capture_output=True,
                         text=True, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith(os.path.join(str(tmp_path), pkg, "libmdx.so"))
    assert (tmp_path / pkg / "libmdx.so").exists()


def test_stale_library_is_detected(tmp_path, monkeypatch):
    """A source newer than the built library marks it stale."""
    from paper_2503_20541_amd import build
    lib = tmp_path / "libmdx.so"
    src = tmp_path / "k.hip"
    src.write_text("//")
    lib.write_text("")
    os.utime(lib, (1000, 1000))
    os.utime(src, (2000, 2000))
    monkeypatch.setattr(build, "LIB", str(lib))
    monkeypatch.setattr(build, "_inputs", lambda: [str(src)])
    assert build.is_stale()
    os.utime(lib, (3000, 3000))
    assert not build.is_stale()
    lib.unlink()
    assert build.is_stale()
