"""HIP graph capture of the launch-bound calls: the small bubble (N = 31, N_q = 201, the size
where launch overhead matters) and a multiloop step over two ragged parameter points are
captured after one warm-up call (workspace allocated, grids cached; the library records its
internal streams into the capture through events), then replayed.  Every replay -- with eager
work and synchronisations between the replays -- equals the eager result bit for bit (the
forward kernels use no atomics), and the replay time is reported beside the eager time.
"""
import time

import numpy as np
import pytest
import torch

from workload import seed_noise

pytestmark = pytest.mark.gpu

CL = ("K1", "K2", "K2p", "K3")


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _seed(K, n, nq, U=1.0, T=0.1):
    g, q, P = K.Grid(n), K.Quad(nq), K.Propagator(1.0, T)
    bare = K.Vertex(g, U)
    noise = seed_noise(n, 0)
    chans = []
    for r in range(3):
        c = K.Channel(1.0, *[to_dev(noise[r][x]) for x in CL])
        c.K1 = c.K1 + K.bubble(r, bare, bare, P, q, class_mask=K.K1).K1
        chans.append(c)
    return K.Vertex(g, U, chans), P, q


def _warm(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()


def _time(fn, reps=20):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


@pytest.mark.parametrize("precision", [0, 1])
def test_small_bubble_replays_from_a_graph(precision):
    K = _K()
    n, nq = 31, 201
    V, P, q = _seed(K, n, nq)
    ref = K.bubble(0, V, V, P, q, precision=precision)
    out = K.alloc_channel(n)
    run = lambda: K.bubble(0, V, V, P, q, precision=precision, out=out)  # noqa: E731
    _warm(run)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for rep in range(3):
        for x in CL:
            getattr(out, x).fill_(float(rep + 1))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for x in CL:
            assert torch.equal(getattr(out, x), getattr(ref, x)), (rep, x)
    t_eager = _time(run)
    t_graph = _time(g.replay)
    print(f"bubble n={n} nq={nq} precision={precision}: eager {t_eager * 1e3:.3f} ms, graph replay "
          f"{t_graph * 1e3:.3f} ms", flush=True)
    for x in CL:
        assert torch.equal(getattr(out, x), getattr(ref, x))


def test_multiloop_step_replays_from_a_graph():
    K = _K()
    pts = [(9, 31, 0.5, 0.1), (15, 45, 1.0, 0.05)]
    Vs, Ps, qs = [], [], []
    for n, nq, U, T in pts:
        V, P, q = _seed(K, n, nq, U, T)
        Vs.append(V)
        Ps.append(P)
        qs.append(q)
    ref = K.mloop_step(Vs, Ps, qs, 3)
    box = {}

    def run():
        box["out"] = K.mloop_step(Vs, Ps, qs, 3)

    _warm(run)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    out = box["out"]
    for rep in range(3):
        for p in range(2):
            for ell in range(3):
                for r in range(3):
                    for x in CL:
                        getattr(out[p][ell][r], x).fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for p in range(2):
            for ell in range(3):
                for r in range(3):
                    for x in CL:
                        assert torch.equal(getattr(out[p][ell][r], x), getattr(ref[p][ell][r], x)), (rep, p, ell, r, x)
    t_eager = _time(run, 5)
    t_graph = _time(g.replay, 5)
    print(f"multiloop step, two points (n = 9, 15), orders <= 3: eager {t_eager * 1e3:.2f} ms, graph replay "
          f"{t_graph * 1e3:.2f} ms", flush=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_bubble_tune_keeps_the_result(precision):
    """The autotuner picks one of its candidate batches, the context applies it to later calls
    with omega_batch = 0, and the result does not depend on the batch (bit for bit)."""
    K = _K()
    n, nq = 21, 61
    V, P, q = _seed(K, n, nq)
    nb, ms = K.bubble_tune(1, V, V, P, q, precision=precision)
    assert nb in {(n + p - 1) // p for p in (1, 2, 3, 4, 6, 8, 12, 16)} and ms > 0
    auto = K.bubble(1, V, V, P, q, precision=precision)
    for b in (1, 5, n):
        ref = K.bubble(1, V, V, P, q, precision=precision, omega_batch=b)
        for x in CL:
            assert torch.equal(getattr(auto, x), getattr(ref, x)), (b, x)
