"""CPU tests of host-side logic: seeded inputs, workload definitions, bench guard rails."""
import os
import subprocess
import sys

import numpy as np

from workload import CONFIGS, MULTILOOP_POINTS, class_shape, complex_noise, random_channel, seed_noise

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_noise_is_seeded_and_ordered():
    a = seed_noise(5, 0)
    b = seed_noise(5, 0)
    for r in range(3):
        for c in ("K1", "K2", "K2p", "K3"):
            assert a[r][c].shape == class_shape(c, 5)
            assert np.array_equal(a[r][c], b[r][c])
    # one generator drawn in the order channel a, p, t x K1, K2, K2', K3
    rng = np.random.default_rng(0)
    first = complex_noise(rng, class_shape("K1", 5))
    assert np.array_equal(first, a[0]["K1"])
    assert abs(np.std(a[0]["K3"].real) - 1e-3) < 1e-4


def test_complex_noise_layout_matches_pairs_of_normals():
    rng = np.random.default_rng(3)
    x = complex_noise(rng, (4, 3), 2.0)
    rng = np.random.default_rng(3)
    z = rng.standard_normal((4, 3, 2))
    assert np.array_equal(x, 2.0 * (z[..., 0] + 1j * z[..., 1]))


def test_workloads():
    w = CONFIGS["bubble_a_n201"]
    assert (w.N, w.Nq, w.U, w.T) == (201, 2001, 1.0, 0.1)
    assert len(MULTILOOP_POINTS) == 12 and {p[2] for p in MULTILOOP_POINTS} == {51, 101, 151, 201}
    rc = random_channel(3, 1)
    assert set(rc) == {"K1", "K2", "K2p", "K3"}


def test_bench_rejects_more_than_one_gpu():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2 and "one GPU" in res.stderr


def test_bench_flop_count():
    sys.path.insert(0, ROOT)
    import bench
    assert abs(bench.algorithmic_flops(201, 2001) / 1e12 - 16.8053) < 1e-3
    assert abs(bench.algorithmic_flops(31, 201) / 1e9 - 6.5337) < 1e-3


def test_bench_traffic_is_tied_to_the_measured_kernel_source():
    """The roofline traffic is reported only for the split GEMM source it was measured on: the
    digest reads that kernel's own section of the kernel file, and a different digest (any edit
    of the kernel) turns the traffic off."""
    sys.path.insert(0, ROOT)
    import bench
    d = bench.kernel_src_digest()
    assert len(d) == 16 and all(c in "0123456789abcdef" for c in d)
    m = bench.MEASURED_TRAFFIC["zgemm_f32_kernel"]
    got = bench.measured_traffic("zgemm_f32_kernel", m["n"], m["nq"], m["omega_batch"])
    if m["src"] == d:
        assert got == round(m["read_bytes"] + m["write_bytes"], 0)
    else:
        assert got is None
    assert bench.measured_traffic("zgemm_f32_kernel", m["n"] + 2, m["nq"], m["omega_batch"]) is None
    assert bench.measured_traffic("zgemm_f64_kernel", m["n"], m["nq"], m["omega_batch"]) is None
