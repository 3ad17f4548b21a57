"""CPU check of the gfx950 code generated from the HIP sources: no scalar-cache writes
(scalar stores, scalar atomics, scalar cache write-back), no packed FP32 VALU ops, and
atomics only as vector global atomics (FP64 ones as native adds)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def isa(tmp_path_factory):
    out = tmp_path_factory.mktemp("isa") / "kernels.s"
    src = os.path.join(ROOT, "paper_2405_20996_amd", "csrc", "kqft_kernels.hip")
    cmd = ["/opt/rocm/bin/hipcc", "-S", "--offload-device-only", "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2405_20996_amd", "csrc"),
           src, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def test_no_scalar_memory_writes(isa):
    bad = re.findall(r"^\s+(s_store\w*|s_atomic\w*|s_dcache_wb\w*|s_buffer_store\w*|s_scratch_store\w*)", isa, re.M)
    assert not bad, sorted(set(bad))


def test_no_packed_fp32(isa):
    assert not re.search(r"v_pk_(fma|add|mul)_f32", isa)


def test_atomics_are_vector_global(isa):
    """FP64 atomics are native vector global adds (no compare-and-swap loops); the integer
    atomics of the adaptive work list are vector global too."""
    ops = set(re.findall(r"\b((?:global|flat|buffer|ds)_atomic_\w+)", isa))
    assert ops <= {"global_atomic_add_f64", "global_atomic_add", "global_atomic_smax"}, ops
