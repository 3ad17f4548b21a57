"""CPU checks of the C ABI library: it builds for gfx950, loads, and exports every
symbol declared in include/kqft.h.  No compute call is made without a GPU."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kqft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kqft_[a-z_]+)\s*\(", src)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for n in ("kqft_bubble", "kqft_sde", "kqft_mloop_step", "kqft_bubble_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2405_20996_amd import kqft as K
    if not os.path.exists(K.LIB_PATH):
        from paper_2405_20996_amd import build
        build.build()
    lib = K.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2405_20996_amd import kqft as K
    monkeypatch.setattr(K, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(K, "_lib", None)
    import pytest
    with pytest.raises(RuntimeError):
        K.lib()


def test_header_is_plain_c():
    """include/kqft.h compiles as strict C99 (a C ABI: no C++ types in the signatures)."""
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        with open(src, "w") as f:
            f.write('#include "kqft.h"\nint main(void) { return 0; }\n')
        res = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                              os.path.join(ROOT, "include"), "-c", src, "-o", os.path.join(d, "t.o")],
                             capture_output=True, text=True)
        assert res.returncode == 0, res.stderr


STRUCTS = {  # C typedef -> ctypes class of the binding
    "kqft_grid": "KqftGrid", "kqft_quad": "KqftQuad", "kqft_chvert": "KqftChvert", "kqft_vertex": "KqftVertex",
    "kqft_propagator": "KqftPropagator", "kqft_chout": "KqftChout", "kqft_opts": "KqftOpts",
    "kqft_mgrid": "KqftMGrid", "kqft_mvertex": "KqftMVertex", "kqft_mprop": "KqftMProp",
    "kqft_adapt_info": "KqftAdaptInfo", "kqft_flow_opts": "KqftFlowOpts", "kqft_flow_info": "KqftFlowInfo",
    "kqft_parquet_opts": "KqftParquetOpts",
}


def test_binding_structs_match_the_header_layout():
    """Every struct of include/kqft.h has a ctypes twin in the binding with the same size and
    the same field names at the same offsets (a C program compiled with gcc prints them)."""
    import ctypes
    import subprocess
    import tempfile
    from paper_2405_20996_amd import kqft as K
    src = open(os.path.join(ROOT, "include", "kqft.h")).read()
    declared = set(re.findall(r"}\s*(kqft_[a-z_]+)\s*;", src))
    assert declared == set(STRUCTS), declared ^ set(STRUCTS)
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kqft.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(K, pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field in cls._fields_:
            lines.append(f'  printf("{cname} {field[0]} %zu\\n", offsetof({cname}, {field[0]}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(c, "w").write("\n".join(lines) + "\n")
        res = subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                             capture_output=True, text=True)
        assert res.returncode == 0, res.stderr
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, pyname in STRUCTS.items():
        cls = getattr(K, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field in cls._fields_:
            assert got[(cname, field[0])] == getattr(cls, field[0]).offset, (cname, field[0])
