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
