"""Parity at the full workload sizes, in the launch configuration the benchmark times.

At these sizes the oracle evaluates sampled outputs one by one (the bubble at random
(w, v, v') blocks, chi at a few transfer frequencies); the FP64 GPU path must agree to
1e-12 and the split-FP32 path to 1e-6, relative to the max-norm of the full GPU FP64
array of the same class.
"""
import numpy as np
import pytest
import torch

import oracle as O
from workload import seed_noise

pytestmark = pytest.mark.gpu

CL = ("K1", "K2", "K2p", "K3")


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def seeded(n, nq, U, T, noise, D=1.0):
    """Oracle and GPU seed vertices: each side its own PT2 K1, the same noise."""
    K = _K()
    og, oq, op = O.Grid(n), O.Quad(nq), O.Prop(D, T)
    ov = O.seeded_vertex(og, U, op, oq, noise)
    g, q, P = K.Grid(n), K.Quad(nq), K.Propagator(D, T)
    bare = K.Vertex(g, U)
    chans = []
    for r in range(3):
        k1 = K.bubble(r, bare, bare, P, q, class_mask=K.K1).K1
        c = K.Channel(1.0, *[to_dev(noise[r][x]) for x in CL])
        c.K1 = c.K1 + k1
        chans.append(c)
    return ov, K.Vertex(g, U, chans), (og, oq, op), (g, q, P)


def sample_points(n, m, seed):
    rng = np.random.default_rng(seed)
    pts = np.stack([np.full(m, 8), rng.integers(0, n, m), rng.integers(0, n, m), rng.integers(0, n, m)], 1)
    pts[:4, 0] = [1, 2, 4, 8]
    pts[4:8] = [[8, 0, 0, 0], [8, n - 1, n - 1, n - 1], [2, n // 2, n - 1, 0], [4, 0, 0, n // 2]]
    return pts


def check_points(out, ref_full_max, pts, ref, tol):
    worst = 0.0
    for p, r_ in zip(pts, ref):
        cls, iw, i, j = (int(x) for x in p)
        if cls == 8:
            gv, name = out.K3[:, iw, i, j], "K3"
        elif cls == 2:
            gv, name = out.K2[:, iw, i], "K2"
        elif cls == 4:
            gv, name = out.K2p[:, iw, j], "K2p"
        else:
            gv, name = out.K1[:, iw], "K1"
        worst = max(worst, np.abs(gv.cpu().numpy() - r_).max() / ref_full_max[name])
    assert worst < tol, worst


def test_headline_workload_n201_sampled_parity():
    """Channel-a bubble at N = 201, Nq = 2001 (U = 1, T = 0.1) in the benchmark's launch
    configuration (three batches of 67 transfer frequencies, gathers and GEMMs in sequence)."""
    K = _K()
    n, nq = 201, 2001
    noise = seed_noise(n, 0)
    ov, kv, (og, oq, op), (g, q, P) = seeded(n, nq, 1.0, 0.1, noise)
    pts = sample_points(n, 48, 3)
    ref = O.bubble_points(0, ov, ov, op, oq, pts)
    out64 = K.bubble(0, kv, kv, P, q, omega_batch=67)
    torch.cuda.synchronize()
    mx = {c: float(getattr(out64, c).abs().max()) for c in CL}
    check_points(out64, mx, pts, ref, 1e-12)
    del out64
    out32 = K.bubble(0, kv, kv, P, q, precision=K.SPLIT_FP32, omega_batch=67)
    torch.cuda.synchronize()
    check_points(out32, mx, pts, ref, 1e-6)


@pytest.mark.parametrize("U", [0.5, 1.0, 2.0])
def test_three_channel_workload_n101(U):
    """All three channels at N = 101, Nq = 1001, T = 0.05: sampled bubble outputs of each
    channel; the self-energy in full and chi at five transfer frequencies on the seeded vertex."""
    K = _K()
    n, nq, T = 101, 1001, 0.05
    noise = seed_noise(n, 0)
    ov, kv, (og, oq, op), (g, q, P) = seeded(n, nq, U, T, noise)
    for r in range(3):
        pts = sample_points(n, 24, 10 + r)
        ref = O.bubble_points(r, ov, ov, op, oq, pts)
        out = K.bubble(r, kv, kv, P, q)
        torch.cuda.synchronize()
        mx = {c: float(getattr(out, c).abs().max()) for c in CL}
        check_points(out, mx, pts, ref, 1e-12)
        del out
    sig, chi = K.sde(kv, P, q, q)
    torch.cuda.synchronize()
    ref_sig = O.sde(ov, op, oq, oq)
    s = sig.cpu().numpy()
    assert np.abs(s - ref_sig).max() < 1e-12 * np.abs(ref_sig).max()
    iws = [0, 25, 50, 51, 100]
    ref_chi = O.chi_points(ov, op, oq, iws)
    c = chi.cpu().numpy()[:, iws]
    assert np.abs(c - ref_chi).max() < 1e-12 * np.abs(ref_chi).max()


def test_three_channel_pipeline_n31():
    """The composite step of the three-channel workload at a size where the oracle computes
    every bubble in full: gamma'_r = B_r(Gamma, Gamma) for r = a, p, t, Gamma' = Gamma_0 +
    sum_r gamma'_r, then Sigma(Gamma') and chi(Gamma')."""
    K = _K()
    n, nq, U, T = 31, 201, 1.0, 0.05
    noise = seed_noise(n, 0)
    ov, kv, (og, oq, op), (g, q, P) = seeded(n, nq, U, T, noise)
    ochans, kchans = [], []
    for r in range(3):
        ref = O.bubble(r, ov, ov, op, oq)
        out = K.bubble(r, kv, kv, P, q)
        torch.cuda.synchronize()
        for c in CL:
            a, b = getattr(out, c).cpu().numpy(), getattr(ref, c)
            assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
        ochans.append(ref)
        kchans.append(out)
    ov2 = O.Vertex(og, U, ochans)
    kv2 = K.Vertex(g, U, kchans)
    sig, chi = K.sde(kv2, P, q, q)
    torch.cuda.synchronize()
    ref_sig = O.sde(ov2, op, oq, oq)
    ref_chi = O.chi(ov2, op, oq)
    assert np.abs(sig.cpu().numpy() - ref_sig).max() < 1e-12 * np.abs(ref_sig).max()
    assert np.abs(chi.cpu().numpy() - ref_chi).max() < 1e-12 * np.abs(ref_chi).max()
    # the scalar retarded susceptibility of the D combination stays finite and the X one is enhanced
    cx = O.chi_scalar(chi.cpu().numpy()[0])
    assert np.all(np.isfinite(cx))


def test_headline_workload_n201_sde_and_chi():
    """Self-energy (in full) and chi (at five transfer frequencies) of the headline vertex,
    N = 201, Nq = 2001 for both the Phi bubble and the loop, FP64."""
    K = _K()
    n, nq = 201, 2001
    noise = seed_noise(n, 0)
    ov, kv, (og, oq, op), (g, q, P) = seeded(n, nq, 1.0, 0.1, noise)
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sig, chi = K.sde(kv, P, q, q)
    torch.cuda.synchronize()
    print(f"sde + chi at n={n}: {time.perf_counter() - t0:.2f} s", flush=True)
    ref_sig = O.sde(ov, op, oq, oq)
    s = sig.cpu().numpy()
    assert np.abs(s - ref_sig).max() < 1e-12 * np.abs(ref_sig).max()
    iws = [0, 50, 100, 101, 200]
    ref_chi = O.chi_points(ov, op, oq, iws)
    c = chi.cpu().numpy()[:, iws]
    assert np.abs(c - ref_chi).max() < 1e-12 * np.abs(ref_chi).max()


@pytest.mark.parametrize("r", [1, 2])
def test_chi_of_the_p_and_t_channels_at_n101(r):
    """kqft_chi in the p and t channels of the N = 101, Nq = 1001 seeded vertex (U = 1, T = 0.05),
    FP64, against the oracle at four transfer frequencies (the edges and the middle)."""
    K = _K()
    n, nq = 101, 1001
    noise = seed_noise(n, 0)
    ov, kv, (og, oq, op), (g, q, P) = seeded(n, nq, 1.0, 0.05, noise)
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chi = K.chi(r, kv, P, q)
    torch.cuda.synchronize()
    print(f"chi channel {r} at n={n}, nq={nq}: {time.perf_counter() - t0:.2f} s", flush=True)
    iws = [0, 50, 51, 100]
    ref = O.chi_channel(r, ov, op, oq, iws)
    c = chi.cpu().numpy()[:, iws]
    assert np.abs(c - ref).max() < 1e-12 * np.abs(ref).max()
