"""kqft_chi_noalloc (the allocation-free susceptibility) against kqft_chi through the C ABI:
two calls in a row on the same device, the second with a smaller input, each equal to the
allocating entry point's result to 1e-12 (FP64); sizes beyond the static scratch rejected."""
import numpy as np
import pytest
import torch

from workload import random_channel

pytestmark = pytest.mark.gpu

D, T, U = 1.0, 0.1, 0.8
CL = ("K1", "K2", "K2p", "K3")


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def _vertex(K, n, seeds, coefs=(1.0, 0.8, 0.6)):
    chans = [random_channel(n, s, 0.2) for s in seeds]
    return K.Vertex(K.Grid(n), U, [K.Channel(c, *[torch.from_numpy(ch[x]).to("cuda") for x in CL])
                                   for c, ch in zip(coefs, chans)])


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def test_chi_noalloc_matches_chi_two_calls_second_smaller():
    K = _K()
    cases = [(21, 61, (1, 2, 3), 0), (11, 23, (4, 5, 6), 2)]  # the second call smaller
    for n, nq, seeds, r in cases:
        V = _vertex(K, n, seeds)
        P, q = K.Propagator(D, T), K.Quad(nq)
        ref = K.chi(r, V, P, q)
        out = torch.full((2, n, 16), float("nan"), dtype=torch.complex128, device="cuda")
        K.chi_noalloc(r, V, P, q, out)
        torch.cuda.synchronize()
        e = _rel(out, ref)
        print(f"n={n} nq={nq} channel {r}: chi_noalloc vs chi {e:.2e}", flush=True)
        assert e < 1e-12, (n, nq, r, e)


def test_chi_noalloc_every_channel_and_a_bare_vertex():
    """Every channel, one with the other channels inactive (no tables), and the algebraic grid."""
    K = _K()
    n, nq = 9, 31
    V = _vertex(K, n, (7, 8, 9))
    for r in range(3):
        ref = K.chi(r, V, K.Propagator(D, T), K.Quad(nq))
        out = torch.zeros((2, n, 16), dtype=torch.complex128, device="cuda")
        K.chi_noalloc(r, V, K.Propagator(D, T), K.Quad(nq), out)
        assert _rel(out, ref) < 1e-12, r
    bare = K.Vertex(K.Grid(n, map=1), U)
    ref = K.chi(1, bare, K.Propagator(D, T), K.Quad(nq, map=1))
    out = torch.zeros((2, n, 16), dtype=torch.complex128, device="cuda")
    K.chi_noalloc(1, bare, K.Propagator(D, T), K.Quad(nq, map=1), out)
    assert _rel(out, ref) < 1e-12


def test_chi_noalloc_rejects_sizes_beyond_the_scratch():
    K = _K()
    n = 41  # two other-channel tables of n^3 + 2n^2 + n records of 512 B exceed 64 MiB
    V = _vertex(K, n, (1, 2, 3))
    out = torch.zeros((2, n, 16), dtype=torch.complex128, device="cuda")
    with pytest.raises(K.KqftError, match="static maximum"):
        K.chi_noalloc(0, V, K.Propagator(D, T), K.Quad(21), out)
