"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: FP64 path within 1e-12 relative to the max-norm of each output array (the
summation order differs; every kernel computes in FP64), split-FP32 path within
1e-6.  Sizes span several 64-wide GEMM tiles with ragged tails in both the
output dimension (4(n+1)) and the contraction (4 nq).
"""
import numpy as np
import pytest
import torch

import oracle as O
from workload import random_channel, seed_noise

pytestmark = pytest.mark.gpu

D, T, U = 1.0, 0.1, 1.0


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def to_dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def make_pair(n, seeds, r0=0.7, coefs=(1.0, 0.8, 0.6), amp=0.3):
    """Random vertex with every class of every channel non-zero, on both sides."""
    K = _K()
    chans = [random_channel(n, s, amp) for s in seeds]
    ov = O.Vertex(O.Grid(n), r0, [O.Channel(c, ch["K1"], ch["K2"], ch["K2p"], ch["K3"]) for c, ch in zip(coefs, chans)])
    kv = K.Vertex(K.Grid(n), r0, [K.Channel(c, *[to_dev(ch[x]) for x in K.CLASSES]) for c, ch in zip(coefs, chans)])
    return ov, kv


def compare(out, ref, tol, classes=("K1", "K2", "K2p", "K3")):
    for name in classes:
        a = getattr(out, name).cpu().numpy()
        b = getattr(ref, name)
        e = rel(a, b)
        assert e < tol, f"{name}: relative error {e:.3e}"


@pytest.mark.parametrize("r", [0, 1, 2])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("n,nq", [(11, 23), (37, 67)])
def test_bubble_fp64_matches_oracle(r, kind, n, nq):
    K = _K()
    ovL, kvL = make_pair(n, (11, 12, 13))
    ovR, kvR = make_pair(n, (21, 22, 23), r0=-0.4, coefs=(0.9, 1.0, 1.1))
    q = (O.Quad(nq, 0, 20.0, 1.0), K.Quad(nq))
    ref = O.bubble(r, ovL, ovR, O.Prop(D, T), q[0], kind)
    out = K.bubble(r, kvL, kvR, K.Propagator(D, T), q[1], pi_kind=kind, omega_batch=5)
    torch.cuda.synchronize()
    compare(out, ref, 1e-12)


def test_bubble_with_dynamic_self_energy_and_infinite_quadrature():
    K = _K()
    n, nq = 15, 41
    ovL, kvL = make_pair(n, (31, 32, 33))
    sg = O.Grid(21)
    sn = sg.nodes()
    SigR = 0.3 * sn / (sn * sn + 4) - 0.2j / (1 + sn * sn)
    op = O.Prop(D, 0.05, eps=0.2, sigma_grid=sg, SigR=SigR)
    kp = K.Propagator(D, 0.05, eps=0.2, sigma_grid=K.Grid(21), SigR=to_dev(SigR))
    ref = O.bubble(1, ovL, ovL, op, O.Quad(nq, 1, 0.0, 1.0), 0)
    out = K.bubble(1, kvL, kvL, kp, K.Quad(nq, K.QUAD_TAN_INFINITE, 0.0, 1.0))
    torch.cuda.synchronize()
    compare(out, ref, 1e-12)


def test_class_mask_and_beta_accumulate():
    K = _K()
    n, nq = 13, 29
    ovL, kvL = make_pair(n, (41, 42, 43))
    ref = O.bubble(2, ovL, ovL, O.Prop(D, T), O.Quad(nq))
    P, q = K.Propagator(D, T), K.Quad(nq)
    out = K.alloc_channel(n)
    K.bubble(2, kvL, kvL, P, q, class_mask=K.K1 | K.K2P, out=out)
    K.bubble(2, kvL, kvL, P, q, class_mask=K.K1 | K.K2P, out=out, beta=1)
    torch.cuda.synchronize()
    assert rel(out.K1.cpu().numpy(), 2 * ref.K1) < 1e-12
    assert rel(out.K2p.cpu().numpy(), 2 * ref.K2p) < 1e-12
    assert float(out.K3.abs().max()) == 0.0 and float(out.K2.abs().max()) == 0.0
    only = K.bubble(2, kvL, kvL, P, q, class_mask=K.K1)
    torch.cuda.synchronize()
    assert rel(only.K1.cpu().numpy(), ref.K1) < 1e-12


def _seeded(n, nq, U=U, Tl=T):
    """Each side computes its own PT2 K1 seed; the noise is shared."""
    K = _K()
    noise = seed_noise(n, 0)
    og, oq, op = O.Grid(n), O.Quad(nq), O.Prop(D, Tl)
    ov = O.seeded_vertex(og, U, op, oq, noise)
    g, q, P = K.Grid(n), K.Quad(nq), K.Propagator(D, Tl)
    bare = K.Vertex(g, U)
    chans = []
    for r in range(3):
        k1 = K.bubble(r, bare, bare, P, q, class_mask=K.K1).K1
        c = K.Channel(1.0, *[to_dev(noise[r][x]) for x in K.CLASSES])
        c.K1 = c.K1 + k1
        chans.append(c)
    return ov, K.Vertex(g, U, chans), (og, oq, op), (g, q, P)


def test_config1_bubble_a_fp64_and_split():
    """n = 31 transfer/fermionic points, 201 quadrature nodes, channel a, seeded vertex."""
    K = _K()
    ov, kv, (og, oq, op), (g, q, P) = _seeded(31, 201)
    for r in range(3):
        assert rel(kv.ch[r].K1.cpu().numpy(), ov.ch[r].K1) < 1e-12
    ref = O.bubble(0, ov, ov, op, oq)
    out = K.bubble(0, kv, kv, P, q)
    torch.cuda.synchronize()
    compare(out, ref, 1e-12)
    out32 = K.bubble(0, kv, kv, P, q, precision=K.SPLIT_FP32)
    torch.cuda.synchronize()
    compare(out32, ref, 1e-6)
    # overlapped gather/GEMM schedule and small batches: the same FP64 result
    out_s = K.bubble(0, kv, kv, P, q, omega_batch=4, overlap=True)
    torch.cuda.synchronize()
    compare(out_s, ref, 1e-12)


def test_sde_and_chi_match_oracle():
    K = _K()
    n, nq = 21, 81
    ov, kv, (og, oq, op), (g, q, P) = _seeded(n, nq)
    ref_sig = O.sde(ov, op, oq, oq)
    ref_chi = O.chi(ov, op, oq)
    sig, chi = K.sde(kv, P, q, q)
    torch.cuda.synchronize()
    assert rel(sig.cpu().numpy(), ref_sig) < 1e-12
    assert rel(chi.cpu().numpy()[0], ref_chi[0]) < 1e-12
    assert rel(chi.cpu().numpy()[1], ref_chi[1]) < 1e-12


@pytest.mark.parametrize("r", [0, 1, 2])
def test_chi_of_every_channel_matches_oracle(r):
    """kqft_chi in channel r for a vertex with every class of every channel non-zero (so the
    own classes, both tables and the bare part all enter), a ragged quadrature."""
    K = _K()
    n, nq = 13, 37
    ov, kv = make_pair(n, (31, 32, 33), r0=U, amp=0.2)
    ref = O.chi_channel(r, ov, O.Prop(D, T), O.Quad(nq))
    out = K.chi(r, kv, K.Propagator(D, T), K.Quad(nq)).cpu().numpy()
    for c in range(2):
        assert rel(out[c], ref[c]) < 1e-12
    if r == 0:
        _, chi_sde = K.sde(kv, K.Propagator(D, T), K.Quad(nq), K.Quad(nq))
        assert np.array_equal(chi_sde.cpu().numpy(), out)
    with pytest.raises(K.KqftError):
        K.chi(3, kv, K.Propagator(D, T), K.Quad(nq))


@pytest.mark.parametrize("n,nq", [(2, 1), (3, 2), (5, 17)])
def test_chi_edge_sizes(n, nq):
    """kqft_chi at the smallest grids and quadratures (a single node, a single block of pairs)
    in every channel."""
    K = _K()
    ov, kv = make_pair(n, (41, 42, 43), r0=U, amp=0.2)
    for r in range(3):
        ref = O.chi_channel(r, ov, O.Prop(D, T), O.Quad(nq))
        out = K.chi(r, kv, K.Propagator(D, T), K.Quad(nq)).cpu().numpy()
        assert rel(out, ref) < 1e-12, r


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-6)])
def test_mloop_four_loops_matches_oracle(prec, tol):
    """Every order l = 1..4 per channel and class: l = 4 is the first order whose centre term
    reads the left insertion kept from two orders back (the rotation of the stored insertions)."""
    K = _K()
    n, nq = 9, 25
    ov, kv = make_pair(n, (51, 52, 53), r0=U, amp=0.05)
    ref = O.mloop(ov, O.Prop(D, T), O.Quad(nq), 4)
    out = K.mloop_step([kv], [K.Propagator(D, T)], [K.Quad(nq)], 4, precision=prec)
    torch.cuda.synchronize()
    for ell in range(4):
        for r in range(3):
            compare(out[0][ell][r], ref[ell][r], tol)


def test_mloop_ragged_points():
    """Three points of different grids, quadratures, U and T in one call, orders l = 1..4."""
    K = _K()
    pts = [(7, 19, 0.5, 0.1), (11, 31, 1.5, 0.01), (5, 13, 1.0, 0.05)]
    kvs, Ps, qs, refs = [], [], [], []
    for i, (n, nq, Ul, Tl) in enumerate(pts):
        ov, kv = make_pair(n, (60 + i, 70 + i, 80 + i), r0=Ul, amp=0.05)
        refs.append(O.mloop(ov, O.Prop(D, Tl), O.Quad(nq), 4))
        kvs.append(kv)
        Ps.append(K.Propagator(D, Tl))
        qs.append(K.Quad(nq))
    out = K.mloop_step(kvs, Ps, qs, 4)
    torch.cuda.synchronize()
    for p in range(len(pts)):
        for ell in range(4):
            for r in range(3):
                compare(out[p][ell][r], refs[p][ell][r], 1e-12)


def test_invalid_arguments_raise():
    K = _K()
    n = 5
    _, kv = make_pair(n, (1, 2, 3))
    with pytest.raises(K.KqftError):
        K.bubble(3, kv, kv, K.Propagator(D, T), K.Quad(9))
    with pytest.raises(K.KqftError):
        K.bubble(0, kv, kv, K.Propagator(D, T), K.Quad(0))
    _, kv7 = make_pair(7, (1, 2, 3))
    with pytest.raises(K.KqftError):
        K.bubble(0, kv, kv7, K.Propagator(D, T), K.Quad(9))


@pytest.mark.parametrize("n,nq,batch", [(2, 1, 1), (2, 3, 5), (15, 16, 3), (16, 9, 16), (3, 1, 2)])
def test_bubble_edge_sizes(n, nq, batch):
    """Degenerate and boundary sizes: the smallest grid (n = 2), a single quadrature node,
    a panel height 4(n + 1) of exactly one tile (n = 15) and one row past it (n = 16), batches
    of one and of more transfer frequencies than the grid has; all channels, both paths."""
    K = _K()
    ovL, kvL = make_pair(n, (91, 92, 93))
    ovR, kvR = make_pair(n, (94, 95, 96), r0=0.3)
    P, q = O.Prop(D, T), O.Quad(nq)
    for r in range(3):
        ref = O.bubble(r, ovL, ovR, P, q)
        out = K.bubble(r, kvL, kvR, K.Propagator(D, T), K.Quad(nq), omega_batch=batch)
        out32 = K.bubble(r, kvL, kvR, K.Propagator(D, T), K.Quad(nq), omega_batch=batch, precision=K.SPLIT_FP32)
        torch.cuda.synchronize()
        compare(out, ref, 1e-12)
        compare(out32, ref, 1e-6)
