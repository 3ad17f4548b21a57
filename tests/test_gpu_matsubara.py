"""Matsubara-formalism bubble on the GPU (kqft_bubble_matsubara) against the oracle.

Every channel, random vertices with every class non-zero and a dynamic self-energy in G,
ragged windows (odd bosonic indices drop one summand): all four classes to 1e-12; a vertex
built from two rounds of GPU bubbles against the oracle's; the degenerate smallest boxes;
argument errors; and the time of a larger bubble.
"""
import time

import numpy as np
import pytest
import torch

from oracle import matsubara as MF

pytestmark = pytest.mark.gpu

CL = ("K1", "K2", "K2p", "K3")
T, D = 0.1, 1.0


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _pair(M, N, seed, U=0.8, amp=0.3):
    K = _K()
    rng = np.random.default_rng(seed)
    g = MF.MGrid(M, N, T)
    sh = g.shapes()
    chans = []
    for r in range(3):
        arrs = [amp * (rng.standard_normal(sh[c]) + 1j * rng.standard_normal(sh[c])) for c in CL]
        chans.append((0.7 + 0.2 * r, arrs))
    ov = MF.MVertex(g, U, [MF.MChannel(c, *a) for c, a in chans])
    kv = K.MVertex(K.MGrid(M, N, T), U, [K.Channel(c, *[to_dev(x) for x in a]) for c, a in chans])
    return ov, kv


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("r", [0, 1, 2])
@pytest.mark.parametrize("M,N,Nq", [(5, 6, 9), (0, 1, 1), (2, 1, 3)])
def test_matsubara_bubble_matches_oracle(r, M, N, Nq):
    K = _K()
    oL, kL = _pair(M, N, 10 + r)
    oR, kR = _pair(M, N, 20 + r, U=-0.5)
    Ns = N + 3
    sig = 0.2 * np.exp(1j * np.linspace(0.0, 3.0, 2 * Ns)) - 0.1j
    ref = MF.bubble(r, oL, oR, MF.MProp(D, T, sig), Nq)
    out = K.bubble_matsubara(r, kL, kR, D, Nq, sigma=to_dev(sig))
    torch.cuda.synchronize()
    for x in CL:
        e = _rel(getattr(out, x).cpu().numpy(), getattr(ref, x))
        assert e < 1e-12, (x, e)


def test_matsubara_vertex_from_gpu_bubbles_matches_oracle():
    """Gamma_1 = Gamma_0 + sum_r B_r(Gamma_0, Gamma_0) and Gamma_2 = Gamma_0 + sum_r B_r(Gamma_1,
    Gamma_1) built from GPU bubbles (M = 12, N = 8, Nq = 24) agree with the oracle's."""
    K = _K()
    M, N, Nq, U = 12, 8, 24, 1.0
    og, kg = MF.MGrid(M, N, T), K.MGrid(M, N, T)
    P = MF.MProp(D, T)
    o0 = MF.bare(og, U)
    o1 = MF.combine(og, U, [(r, MF.bubble(r, o0, o0, P, Nq), 1.0) for r in range(3)])
    o2 = [MF.bubble(r, o1, o1, P, Nq) for r in range(3)]
    k0 = K.MVertex(kg, U)
    k1 = K.MVertex(kg, U, [K.bubble_matsubara(r, k0, k0, D, Nq) for r in range(3)])
    k2 = [K.bubble_matsubara(r, k1, k1, D, Nq) for r in range(3)]
    torch.cuda.synchronize()
    for r in range(3):
        for x in CL:
            assert _rel(getattr(k2[r], x).cpu().numpy(), getattr(o2[r], x)) < 1e-12, (r, x)


def test_matsubara_invalid_arguments_raise():
    K = _K()
    _, kv = _pair(2, 2, 1)
    with pytest.raises(K.KqftError):
        K.bubble_matsubara(3, kv, kv, D, 4)
    with pytest.raises(K.KqftError):
        K.bubble_matsubara(0, kv, kv, D, 0)
    _, kw = _pair(2, 3, 1)
    with pytest.raises(K.KqftError):
        K.bubble_matsubara(0, kv, kw, D, 4)


def test_matsubara_bubble_time():
    """M = 100, N = 100, Nq = 200: (2N + 1) x 2Nq x (2N + 1) complex products for 201 bosonic
    frequencies and two spin combinations (52 GFLOP); all three channels, each sampled at five
    bosonic frequencies (both box edges, the centre, an odd and an even index) against the
    oracle to 1e-12."""
    K = _K()
    M, N, Nq = 100, 100, 200
    ov, kv = _pair(M, N, 5, amp=0.05)
    ms = [-M, -37, 0, 64, M]
    K.bubble_matsubara(0, kv, kv, D, Nq)
    torch.cuda.synchronize()
    for r in range(3):
        t0 = time.perf_counter()
        out = K.bubble_matsubara(r, kv, kv, D, Nq)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flop = 8.0 * (2 * N + 1) ** 2 * 2 * Nq * 2 * (2 * M + 1)
        print(f"Matsubara bubble r={r} M={M} N={N} Nq={Nq}: {dt * 1e3:.1f} ms, {flop / dt / 1e12:.1f} TFLOP/s "
              f"(algorithmic)", flush=True)
        ref = MF.bubble(r, ov, ov, MF.MProp(D, T), Nq, ms=ms)
        im = [m + M for m in ms]
        for x in CL:
            a, b = getattr(out, x).cpu().numpy()[:, im], getattr(ref, x)[:, im]
            e = _rel(a, b)
            assert e < 1e-12, (r, x, e)


def test_matsubara_sde_matches_oracle():
    """Sigma from the Matsubara SDE (Phi = B_a(Gamma_0, Gamma) on the GPU, then the loop) for a
    random vertex and a dynamic self-energy in G (M = N + Nl keeps every term)."""
    K = _K()
    M, N, Nq, Nl = 12, 4, 10, 8
    ov, kv = _pair(M, N, 7, U=1.0)
    Ns = 6
    sig = 0.1 * np.exp(1j * np.linspace(0.0, 2.0, 2 * Ns)) - 0.05j
    ref = MF.sde(ov, MF.MProp(D, T, sig), Nq, Nl)
    out = K.sde_matsubara(kv, D, Nq, Nl, sigma=to_dev(sig)).cpu().numpy()
    assert _rel(out, ref) < 1e-12
    with pytest.raises(K.KqftError):
        K.sde_matsubara(kv, D, Nq, 0)


@pytest.mark.parametrize("alpha,depth,reduce", [(0.5, 0, False), (0.5, 3, False), (1.0, 2, True)])
def test_matsubara_parquet_solver_matches_oracle(alpha, depth, reduce):
    """The Matsubara parquet solver (PT2 start; linear mixing, Anderson acceleration, alpha
    reduction): residuals and final state as the oracle's (M = 12, N = 4, Nq = 12, Nl = 8)."""
    K = _K()
    M, N, Nq, Nl, U, iters = 12, 4, 12, 8, 1.0, 6
    och, osig, ores = MF.parquet_solve(MF.MGrid(M, N, T), U, D, Nq, Nl, alpha=alpha, iterations=iters, depth=depth,
                                       reduce_alpha=reduce)
    kch, ksig, kres = K.parquet_solve_matsubara(K.MGrid(M, N, T), U, D, Nq, Nl, alpha=alpha, max_iterations=iters,
                                                depth=depth, reduce_alpha=reduce)
    torch.cuda.synchronize()
    print(f"alpha={alpha} depth={depth}: residuals {['%.2e' % x for x in kres]}", flush=True)
    assert len(kres) == iters and np.allclose(kres, ores, rtol=1e-9, atol=0)
    for r in range(3):
        for x in CL:
            assert _rel(getattr(kch[r], x).cpu().numpy(), getattr(och[r], x)) < 1e-10, (r, x)
    assert _rel(ksig.cpu().numpy(), osig) < 1e-10
    with pytest.raises(K.KqftError):
        K.parquet_solve_matsubara(K.MGrid(M, N, T), U, D, Nq, Nl, alpha=0.0)


def test_matsubara_parquet_solver_time():
    """M = 96, N = 48, Nq = 96, Nl = 48 (every SDE term inside the boxes), U = 1, eight
    iterations with Anderson depth 3: the time per iteration (six Matsubara bubbles, the SDE
    bubble and loop, the mixing) and a contracting residual."""
    K = _K()
    M, N, Nq, Nl, iters = 96, 48, 96, 48, 8
    K.parquet_solve_matsubara(K.MGrid(M, N, T), 1.0, D, Nq, Nl, max_iterations=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, res = K.parquet_solve_matsubara(K.MGrid(M, N, T), 1.0, D, Nq, Nl, alpha=0.5, max_iterations=iters, depth=3)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    print(f"Matsubara parquet M={M} N={N} Nq={Nq}: {dt * 1e3:.1f} ms per iteration, residuals "
          f"{['%.2e' % x for x in res]}", flush=True)
    assert res[-1] < 0.1 * res[1]


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("Nl", [9, 70])
def test_matsubara_loop_matches_oracle(kind, Nl):
    """kqft_loop_matsubara of a random vertex (every channel and class, bare part) with G, S + G
    Sigma_dot G or G Sigma_dot G, dynamic Sigma.  Nl = 70 puts 140 loop frequencies on the 64
    lanes of a wavefront, so every lane sums several of them before the LDS reduction."""
    K = _K()
    M, N = 8, 5
    ov, kv = _pair(M, N, 13, U=0.7)
    Ns = N + 2
    sig = 0.1 * np.exp(1j * np.linspace(0.0, 2.0, 2 * Ns)) - 0.05j
    dsig = 0.2 * np.exp(-1j * np.linspace(0.0, 1.0, 2 * Ns))
    ref = MF.loop(ov, MF.MProp(1.3, T, sig, dsig), Nl, kind)
    out = K.loop_matsubara(kv, 1.3, Nl, kind, sigma=to_dev(sig), dsigma=to_dev(dsig)).cpu().numpy()
    assert _rel(out, ref) < 1e-12


@pytest.mark.parametrize("r", [0, 1, 2])
def test_matsubara_pidot_bubble_matches_oracle(r):
    K = _K()
    M, N, Nq = 4, 4, 7
    oL, kL = _pair(M, N, 30 + r)
    oR, kR = _pair(M, N, 40 + r, U=-0.4)
    Ns = N + 3
    sig = 0.2 * np.exp(1j * np.linspace(0.0, 3.0, 2 * Ns)) - 0.1j
    dsig = 0.3 * np.exp(-1j * np.linspace(0.0, 2.0, 2 * Ns))
    ref = MF.bubble(r, oL, oR, MF.MProp(D, T, sig, dsig), Nq, 1)
    out = K.bubble_matsubara(r, kL, kR, D, Nq, sigma=to_dev(sig), dsigma=to_dev(dsig), pi_kind=K.PI_DOT)
    torch.cuda.synchronize()
    for x in CL:
        assert _rel(getattr(out, x).cpu().numpy(), getattr(ref, x)) < 1e-12, x


@pytest.mark.parametrize("steps,nloops,katanin,se", [(2, 1, False, 0), (1, 3, True, 3), (1, 2, True, 0)])
def test_matsubara_flow_matches_oracle(steps, nloops, katanin, se):
    """The Matsubara hybridization flow from the PT2 state (Delta 2 -> 1, U = 1, M = 8, N = 3):
    one-loop RK4, three loops with Katanin and self-energy corrections, two loops with Katanin."""
    K = _K()
    M, N, Nq, Nl, U = 8, 3, 8, 6, 1.0
    og = MF.MGrid(M, N, T)
    chans, sig = MF.pt2_state(og, U, 2.0, Nq, Nl)
    rch, rsig = MF.mfrg_flow(og, U, 2.0, 1.0, steps, nloops, Nq, Nl, chans, sig, katanin, se)
    kch = [K.Channel(1.0, *[to_dev(getattr(c, x)) for x in CL]) for c in chans]
    ksig = to_dev(sig)
    K.mfrg_flow_matsubara(K.MGrid(M, N, T), U, 2.0, 1.0, steps, nloops, Nq, Nl, kch, ksig, katanin=katanin,
                          se_iterations=se)
    torch.cuda.synchronize()
    for r in range(3):
        for x in CL:
            b = getattr(rch[r], x)
            if np.abs(b).max() == 0.0:
                assert float(getattr(kch[r], x).abs().max()) == 0.0
                continue
            assert _rel(getattr(kch[r], x).cpu().numpy(), b) < 1e-10, (r, x)
    assert _rel(ksig.cpu().numpy(), rsig) < 1e-10


def test_matsubara_adaptive_flow_matches_oracle():
    """Cash-Karp step control on the Matsubara flow (M = 8, N = 3, two loops, Katanin, Delta
    2 -> 1, tolerances 1e-7 / 1e-5): the same accepted Delta values and rejected steps as the
    oracle, and the same final state to 1e-10."""
    K = _K()
    M, N, Nq, Nl, U = 8, 3, 8, 6, 1.0
    og = MF.MGrid(M, N, T)
    chans, sig = MF.pt2_state(og, U, 2.0, Nq, Nl)
    rinfo = {}
    rch, rsig = MF.mfrg_flow(og, U, 2.0, 1.0, 2, 2, Nq, Nl, chans, sig, True, 0, adaptive=True, atol=1e-7,
                             rtol=1e-5, info=rinfo)
    kch = [K.Channel(1.0, *[to_dev(getattr(c, x)) for x in CL]) for c in chans]
    ksig = to_dev(sig)
    _, _, kinfo = K.mfrg_flow_matsubara(K.MGrid(M, N, T), U, 2.0, 1.0, 2, 2, Nq, Nl, kch, ksig, katanin=True,
                                        adaptive=True, atol=1e-7, rtol=1e-5)
    torch.cuda.synchronize()
    print(f"adaptive Matsubara flow: Delta {np.round(kinfo['lambdas'], 6).tolist()}, rejected {kinfo['rejected']}, "
          f"rhs {kinfo['rhs']}", flush=True)
    assert len(kinfo["lambdas"]) == len(rinfo["lambdas"]) and kinfo["rejected"] == rinfo["rejected"]
    assert np.abs(np.array(kinfo["lambdas"]) - np.array(rinfo["lambdas"])).max() < 1e-12
    # six stages per accepted trial, five per rejected one (its first stage is reused)
    assert kinfo["rhs"] == 6 * (len(rinfo["lambdas"]) - 1) + 5 * rinfo["rejected"]
    for r in range(3):
        for x in CL:
            assert _rel(getattr(kch[r], x).cpu().numpy(), getattr(rch[r], x)) < 1e-10, (r, x)
    assert _rel(ksig.cpu().numpy(), rsig) < 1e-10
    with pytest.raises(K.KqftError):  # step limit
        K.mfrg_flow_matsubara(K.MGrid(M, N, T), U, 2.0, 1.0, 2, 1, Nq, Nl, kch, ksig, adaptive=True, atol=1e-14,
                              rtol=1e-14, max_steps=2)


def test_matsubara_flow_time():
    """M = 48, N = 24, Nq = 48, Nl = 24, U = 1: two RK4 steps of the hybridization flow from the
    PT2 state (Delta 2 -> 1), three loops with Katanin and up to three correction iterations; the
    time per right-hand side and a finite state."""
    K = _K()
    M, N, Nq, Nl, U = 48, 24, 48, 24, 1.0
    og = MF.MGrid(M, N, T)
    chans, sig = MF.pt2_state(og, U, 2.0, Nq, Nl)
    kch = [K.Channel(1.0, *[to_dev(getattr(c, x)) for x in CL]) for c in chans]
    ksig = to_dev(sig)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    K.mfrg_flow_matsubara(K.MGrid(M, N, T), U, 2.0, 1.0, 2, 3, Nq, Nl, kch, ksig, katanin=True, se_iterations=3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"Matsubara flow M={M} N={N} Nq={Nq}, l<=3, Katanin, corrections: {dt * 1e3:.1f} ms for 8 right-hand "
          f"sides ({dt / 8 * 1e3:.1f} ms each)", flush=True)
    assert all(bool(torch.isfinite(getattr(c, x)).all()) for c in kch for x in CL)
    assert bool(torch.isfinite(ksig).all())


@pytest.mark.parametrize("r", [0, 1, 2])
def test_matsubara_bubble_with_analytic_tails_matches_oracle(r):
    """tails = 1: the bare bubble's closed form beyond the window (host digamma/trigamma series)
    and the tail kernel against the oracle (scipy's digamma), random vertices, dynamic Sigma, a
    window that does not cover the boxes; and the window independence for the bare vertex."""
    K = _K()
    M, N, Nq = 5, 4, 3
    oL, kL = _pair(M, N, 50 + r)
    oR, kR = _pair(M, N, 60 + r, U=-0.6)
    Ns = N + 2
    sig = 0.2 * np.exp(1j * np.linspace(0.0, 3.0, 2 * Ns)) - 0.1j
    ref = MF.bubble(r, oL, oR, MF.MProp(D, T, sig), Nq, tails=True)
    out = K.bubble_matsubara(r, kL, kR, D, Nq, sigma=to_dev(sig), tails=True)
    torch.cuda.synchronize()
    for x in CL:
        assert _rel(getattr(out, x).cpu().numpy(), getattr(ref, x)) < 1e-12, x
    k0 = K.MVertex(K.MGrid(M, N, T), 1.0)
    a = K.bubble_matsubara(r, k0, k0, D, 2, tails=True).K1
    b = K.bubble_matsubara(r, k0, k0, D, 400, tails=True).K1
    assert float((a - b).abs().max()) < 1e-13 * float(b.abs().max())
    with pytest.raises(K.KqftError):
        K.bubble_matsubara(r, k0, k0, D, 2, tails=True, pi_kind=K.PI_DOT)


@pytest.mark.parametrize("r", [0, 1, 2])
@pytest.mark.parametrize("M,N,Nq", [(5, 6, 9), (0, 1, 1), (3, 2, 40)])
def test_matsubara_chi_matches_oracle(r, M, N, Nq):
    """chi_r^c(m) for a random vertex (every class and channel non-zero) and a dynamic
    self-energy in G, against the oracle to 1e-12; the largest case spans more pairs per m
    than one workgroup holds."""
    K = _K()
    ov, kv = _pair(M, N, 40 + r)
    Ns = N + 2
    sig = 0.15 * np.exp(1j * np.linspace(0.0, 2.0, 2 * Ns)) - 0.05j
    ref = MF.chi(r, ov, MF.MProp(D, T, sig), Nq)
    out = K.chi_matsubara(r, kv, D, Nq, sigma=to_dev(sig))
    torch.cuda.synchronize()
    e = _rel(out.cpu().numpy(), ref)
    assert e < 1e-12, e


def test_matsubara_chi_errors():
    K = _K()
    _, kv = _pair(2, 2, 3)
    with pytest.raises(K.KqftError):
        K.chi_matsubara(3, kv, D, 4)
    with pytest.raises(K.KqftError):
        K.chi_matsubara(0, kv, D, 0)


def test_matsubara_chi_full_box_time_and_samples():
    """M = N = 100, Nq = 200 (201 bosonic frequencies x 400^2 full-vertex lookups): timing, and
    five bosonic frequencies of every channel against the oracle to 1e-12."""
    K = _K()
    M, N, Nq = 100, 100, 200
    ov, kv = _pair(M, N, 6, amp=0.05)
    ms = [-M, -37, 0, 64, M]
    K.chi_matsubara(0, kv, D, Nq)
    torch.cuda.synchronize()
    for r in range(3):
        t0 = time.perf_counter()
        out = K.chi_matsubara(r, kv, D, Nq)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"Matsubara chi r={r} M={M} N={N} Nq={Nq}: {dt * 1e3:.2f} ms "
              f"({(2 * M + 1) * (2 * Nq) ** 2 / dt / 1e9:.1f} G vertex lookups/s)", flush=True)
        ref = MF.chi(r, ov, MF.MProp(D, T), Nq, ms=ms)
        im = [m + M for m in ms]
        e = _rel(out.cpu().numpy()[:, im], ref[:, im])
        assert e < 1e-12, (r, e)


@pytest.mark.parametrize("r", [0, 1, 2])
def test_matsubara_interaction_regulator_matches_oracle(r):
    """G_0 -> lam G_0 (lam = 0.7): the G G and the S G + G S bubbles (with Sigma and Sigma_dot)
    and the S loop against the oracle to 1e-12; the analytic tails refuse the regulated G_0."""
    K = _K()
    M, N, Nq = 5, 6, 9
    oL, kL = _pair(M, N, 70 + r)
    oR, kR = _pair(M, N, 80 + r, U=-0.5)
    Ns = N + 2
    sig = 0.2 * np.exp(1j * np.linspace(0.0, 3.0, 2 * Ns)) - 0.1j
    dsig = 0.3 * np.exp(-1j * np.linspace(0.0, 2.0, 2 * Ns))
    P = MF.MProp(D, T, sig, dsig, reg=1, lam=0.7)
    for kind in (0, 1):
        ref = MF.bubble(r, oL, oR, P, Nq, kind)
        out = K.bubble_matsubara(r, kL, kR, D, Nq, sigma=to_dev(sig), dsigma=to_dev(dsig), pi_kind=kind, reg=1,
                                 lam=0.7)
        torch.cuda.synchronize()
        for x in CL:
            assert _rel(getattr(out, x).cpu().numpy(), getattr(ref, x)) < 1e-12, (kind, x)
    if r == 0:
        ref = MF.loop(oL, P, 7, 1)
        out = K.loop_matsubara(kL, D, 7, K.LINE_S, sigma=to_dev(sig), dsigma=to_dev(dsig), reg=1, lam=0.7)
        assert _rel(out.cpu().numpy(), ref) < 1e-12
        with pytest.raises(K.KqftError):
            K.bubble_matsubara(0, kL, kR, D, Nq, tails=True, reg=1, lam=0.7)
        with pytest.raises(K.KqftError):
            K.bubble_matsubara(0, kL, kR, D, Nq, reg=1, lam=0.0)


def test_matsubara_interaction_flow_matches_oracle():
    """The Matsubara interaction flow from the PT2 state at lam = 0.5 to lam = 1 (Delta = 1,
    M = 8, N = 3, two loops, Katanin, one RK4 step) against the oracle to 1e-10."""
    K = _K()
    M, N, Nq, Nl, U = 8, 3, 8, 6, 1.0
    og = MF.MGrid(M, N, T)
    chans, sig = MF.pt2_state(og, U, 1.0, Nq, Nl, reg=1, lam=0.5)
    rch, rsig = MF.mfrg_flow(og, U, 0.5, 1.0, 1, 2, Nq, Nl, chans, sig, True, 0, reg=1, Delta=1.0)
    kch = [K.Channel(1.0, *[to_dev(getattr(c, x)) for x in CL]) for c in chans]
    ksig = to_dev(sig)
    _, _, info = K.mfrg_flow_matsubara(K.MGrid(M, N, T), U, 0.5, 1.0, 1, 2, Nq, Nl, kch, ksig, katanin=True,
                                       reg=1, Delta=1.0)
    torch.cuda.synchronize()
    assert np.abs(np.array(info["lambdas"]) - [0.5, 1.0]).max() < 1e-14
    for r in range(3):
        for x in CL:
            b = getattr(rch[r], x)
            if np.abs(b).max() == 0.0:
                continue
            assert _rel(getattr(kch[r], x).cpu().numpy(), b) < 1e-10, (r, x)
    assert _rel(ksig.cpu().numpy(), rsig) < 1e-10
