"""Batched multiloop workload: twelve parameter points U in {0.25, 0.5, 1, 1.5, 2, 3} x
T in {0.01, 0.1}, N cycling through 51, 101, 151, 201 with Nq = 10 N - 9, loop orders
l = 1..4 in all three channels (27 bubbles per point), Pidot from the Delta-flow
single-scale propagator, on the PT2 seed + 1e-3 noise.

Each point runs through kqft_mloop_step on the split-FP32 path; the test reports the
algorithmic throughput over the batch.  Parity: on the points with N <= 151 every order,
channel and class of the split path agrees with the FP64 path to 1e-6 (relative to each
array's max-norm); on the points with N <= 101 the first order (l = 1, the Pidot bubble
of the seed vertex) agrees with the oracle on sampled outputs, FP64 to 1e-12 and split to
1e-6.  Higher orders are checked against the oracle in full at small sizes
(test_gpu_parity.py); at these sizes the oracle cannot build the lower-order insertions
they take as input.
"""
import time

import numpy as np
import pytest
import torch

import oracle as O
from workload import MULTILOOP_POINTS, seed_noise

pytestmark = pytest.mark.gpu

CL = ("K1", "K2", "K2p", "K3")
NLOOPS = 4


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def gpu_seed(K, n, nq, U, T, noise):
    g, q, P = K.Grid(n), K.Quad(nq), K.Propagator(1.0, T)
    bare = K.Vertex(g, U)
    chans = []
    for r in range(3):
        c = K.Channel(1.0, *[to_dev(noise[r][x]) for x in CL])
        c.K1 = c.K1 + K.bubble(r, bare, bare, P, q, class_mask=K.K1).K1
        chans.append(c)
    return K.Vertex(g, U, chans), P, q


def sample_points(n, m, seed):
    rng = np.random.default_rng(seed)
    pts = np.stack([np.full(m, 8), rng.integers(0, n, m), rng.integers(0, n, m), rng.integers(0, n, m)], 1)
    pts[:4, 0] = [1, 2, 4, 8]
    return pts


def sampled_error(out, pts, ref):
    worst = 0.0
    for p, r_ in zip(pts, ref):
        cls, iw, i, j = (int(x) for x in p)
        arr = {8: out.K3, 2: out.K2, 4: out.K2p, 1: out.K1}[cls]
        gv = {8: lambda: arr[:, iw, i, j], 2: lambda: arr[:, iw, i], 4: lambda: arr[:, iw, j],
              1: lambda: arr[:, iw]}[cls]()
        worst = max(worst, float(np.abs(gv.cpu().numpy() - r_).max() / arr.abs().max()))
    return worst


def test_multiloop_batch_twelve_points():
    K = _K()
    noises = {}
    flop, seconds = 0.0, 0.0
    for idx, (U, T, n) in enumerate(MULTILOOP_POINTS):
        nq = 10 * n - 9
        if n not in noises:
            noises[n] = seed_noise(n, 0)
        noise = noises[n]
        print(f"point {idx}: U={U} T={T} n={n} nq={nq}", flush=True)
        V, P, q = gpu_seed(K, n, nq, U, T, noise)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = K.mloop_step([V], [P], [q], NLOOPS, precision=K.SPLIT_FP32)[0]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        f = 27 * 2.0 * n * 8.0 * (4 * n + 4) * 4.0 * nq * (4 * n + 4)
        flop += f
        seconds += dt
        print(f"   split mloop l<=4: {dt * 1e3:.1f} ms, {f / dt / 1e12:.2f} TFLOP/s", flush=True)
        if n <= 151:
            ref = K.mloop_step([V], [P], [q], NLOOPS)[0]
            torch.cuda.synchronize()
            worst = 0.0
            for ell in range(NLOOPS):
                for r in range(3):
                    for x in CL:
                        a, b = getattr(out[ell][r], x), getattr(ref[ell][r], x)
                        worst = max(worst, float((a - b).abs().max() / b.abs().max()))
            print(f"   split vs fp64 (all orders, channels, classes): {worst:.3e}", flush=True)
            assert worst < 1e-6
            if n <= 101:
                og, oq, op = O.Grid(n), O.Quad(nq), O.Prop(1.0, T)
                ov = O.seeded_vertex(og, U, op, oq, noise)
                for r in range(3):
                    pts = sample_points(n, 12, 100 * idx + r)
                    pref = O.bubble_points(r, ov, ov, op, oq, pts, kind=1)
                    e64 = sampled_error(ref[0][r], pts, pref)
                    e32 = sampled_error(out[0][r], pts, pref)
                    assert e64 < 1e-12, (idx, r, e64)
                    assert e32 < 1e-6, (idx, r, e32)
            del ref
        del out, V
        torch.cuda.empty_cache()
    print(f"batch: {flop / 1e15:.3f} PFLOP algorithmic in {seconds:.2f} s of mloop calls = "
          f"{flop / seconds / 1e12:.2f} TFLOP/s", flush=True)
