"""Pins of the oracle's finite-temperature Matsubara formalism (the bubble, loop and SDE of the
paper carried over to discrete Matsubara sums): the bare bubble against its closed form
(digamma functions) with the window's tail, the bubble of every channel against the literal
compound-index sum over internal legs and spins, crossing symmetry of the vertex built from
bubbles, and the second-order self-energy against the spectral representation of the Keldysh
one (the pinned real-frequency oracle), which fixes sign and normalisation across formalisms."""
import numpy as np
import scipy.special as sp

import oracle as O
from oracle import matsubara as MF

T, D, U = 0.1, 1.0, 1.0


def _bare_bubble_closed_form(m, Dl=D, Tl=T):
    """T sum_n G(n + m) G(n) over all n, G = 1/(i nu + i Dl sgn nu): the two regions where
    both frequencies have the same sign give digamma differences, the m mixed terms are summed."""
    m = abs(m)
    d = Dl / (2 * np.pi * Tl)
    c = 1.0 / (2 * np.pi * Tl) ** 2
    same = c * (sp.polygamma(1, 0.5 + d) if m == 0 else (sp.digamma(0.5 + m + d) - sp.digamma(0.5 + d)) / m)
    mixed = sum(1.0 / ((MF.nu(n + m, Tl) + Dl) * (MF.nu(n, Tl) - Dl)) for n in range(-m, 0))
    return -Tl * (2 * same + mixed)


def test_bare_bubble_converges_to_its_closed_form_with_the_tail_of_the_window():
    """The window |2n + 1 + m| <= 2 Nq - 1 misses the tails T sum 1/nu^2 = 1/(2 pi^2 T Nq) to
    leading order: (window sum - infinite sum) Nq -> 1/(2 pi^2 T); the p bubble at particle-hole
    symmetry is minus the a bubble (G odd in nu)."""
    P = MF.MProp(D, T)
    for m in (0, 1, 2, 5, -3):
        exact = _bare_bubble_closed_form(m)
        for Nq in (1000, 8000):
            k = MF.window(0, m, Nq)
            s = MF.pi_r(0, P, m, k).sum()
            assert abs(s.imag) < 1e-15
            assert abs((s.real - exact) * Nq * 2 * np.pi ** 2 * T - 1.0) < 3.0 / Nq ** 0.5
            sp_ = MF.pi_r(1, P, m, MF.window(1, m, Nq)).sum()
            assert abs(sp_ + s) < 1e-12


def _random_vertex(g, seed, amp=0.3):
    rng = np.random.default_rng(seed)
    sh = g.shapes()
    chans = []
    for r in range(3):
        arrs = [amp * (rng.standard_normal(sh[c]) + 1j * rng.standard_normal(sh[c])) for c in MF.CLASSES]
        chans.append(MF.MChannel(0.7 + 0.2 * r, *arrs))
    return MF.MVertex(g, 0.8, chans)


def _literal_bubble(r, L, R, P, Nq, m, n, npr, spins):
    """The bubble of channel r at (m, n, n') and external spins, summed literally over the
    internal legs' frequency (the window) and spins, from the compound-index definitions:
      a: + L(1'4'|32) G(3) G(4) R(3'2'|14),  p: 1/2 L(1'2'|34) G(3) G(4) R(3'4'|12),
      t: - L(4'2'|32) G(3) G(4) R(1'3'|14)."""
    n1p, n2p, n1, n2 = MF.legs_of(r, m, n, npr)
    s1p, s2p, s1, s2 = spins
    tot = 0.0
    for k in MF.window(r, m, Nq):
        for s3 in (0, 1):
            for s4 in (0, 1):
                if r == 0:    # nu4 = nu'' , nu3 = nu'' + omega
                    n4, n3 = k, k + m
                    lv = MF.vertex_legs(L, (s1p, s4, s3, s2), (n1p, n4, n3, n2))
                    rv = MF.vertex_legs(R, (s3, s2p, s1, s4), (n3, n2p, n1, n4))
                    tot += T * lv * P(n3) * P(n4) * rv
                elif r == 1:  # nu3 = nu'', nu4 = omega - nu''
                    n3, n4 = k, m - k - 1
                    lv = MF.vertex_legs(L, (s1p, s2p, s3, s4), (n1p, n2p, n3, n4))
                    rv = MF.vertex_legs(R, (s3, s4, s1, s2), (n3, n4, n1, n2))
                    tot += 0.5 * T * lv * P(n3) * P(n4) * rv
                else:         # nu4 = nu'', nu3 = nu'' + omega
                    n4, n3 = k, k + m
                    lv = MF.vertex_legs(L, (s4, s2p, s3, s2), (n4, n2p, n3, n2))
                    rv = MF.vertex_legs(R, (s1p, s3, s1, s4), (n1p, n3, n1, n4))
                    tot -= T * lv * P(n3) * P(n4) * rv
    return tot


def test_bubble_of_every_channel_is_the_literal_sum_over_internal_legs_and_spins():
    """K1 + K2 + K2' + K3 of the bubble (asymptotic decomposition, diagonalised spin sums) at
    sample outputs equals the literal sum over the internal frequency and spins of random
    vertices (every class of every channel non-zero) with a dynamic self-energy in G."""
    g = MF.MGrid(3, 3, T)
    L, R = _random_vertex(g, 1), _random_vertex(g, 2)
    sig = 0.2 * np.exp(1j * np.linspace(0, 3, 16)) - 0.1j
    P = MF.MProp(D, T, sig)
    Nq = 5
    rng = np.random.default_rng(4)
    for r in range(3):
        b = MF.bubble(r, L, R, P, Nq)
        for _ in range(6):
            m, n, npr = int(rng.integers(-3, 4)), int(rng.integers(-3, 3)), int(rng.integers(-3, 3))
            val = MF.channel_value(b, g, m, n, npr)
            lx = _literal_bubble(r, L, R, P, Nq, m, n, npr, (0, 1, 0, 1))
            ly = _literal_bubble(r, L, R, P, Nq, m, n, npr, (0, 1, 1, 0))
            scale = max(abs(lx), abs(ly))
            assert scale > 1e-3
            assert abs(val[0] - lx) < 1e-13 * scale and abs(val[1] - ly) < 1e-13 * scale, (r, m, n, npr)


def _crossing_residual(V, lim, seed=3):
    rng = np.random.default_rng(seed)
    worst = scale = 0.0
    for _ in range(200):
        n1p, n2p, n1 = rng.integers(-lim, lim, 3)
        n2 = n1p + n2p - n1
        for s in ([0, 1, 0, 1], [0, 1, 1, 0], [0, 0, 0, 0]):
            x = MF.vertex_legs(V, s, (n1p, n2p, n1, n2))
            y = MF.vertex_legs(V, [s[0], s[1], s[3], s[2]], (n1p, n2p, n2, n1))
            worst, scale = max(worst, abs(x + y)), max(scale, abs(x))
    return worst / scale


def test_vertex_from_bubbles_is_crossing_symmetric():
    """Gamma(1'2'|21) = -Gamma(1'2'|12) for Gamma_1 = Gamma_0 + sum_r B_r(Gamma_0, Gamma_0) and for
    Gamma_2 = Gamma_0 + sum_r B_r(Gamma_1, Gamma_1) (legs well inside the box): crossing maps
    the a bubble onto the t bubble and the p bubble onto itself, so this checks the three
    parametrisations, the prefactors and the spin sums together."""
    g = MF.MGrid(12, 8, T)
    P = MF.MProp(D, T)
    g0 = MF.bare(g, U)
    V1 = MF.combine(g, U, [(r, MF.bubble(r, g0, g0, P, 24), 1.0) for r in range(3)])
    assert _crossing_residual(V1, 6) < 1e-14
    V2 = MF.combine(g, U, [(r, MF.bubble(r, V1, V1, P, 24), 1.0) for r in range(3)])
    assert _crossing_residual(V2, 2) < 1e-14


def test_second_order_self_energy_is_the_spectral_representation_of_the_keldysh_one():
    """Sigma^(2)(i nu_n) of the Matsubara SDE equals -1/pi int de Im Sigma^R(e) / (i nu_n - e)
    with Sigma^R the Keldysh oracle's second-order self-energy (same Delta, T, U): the two
    formalisms agree on sign and normalisation, up to the Keldysh grid and the Matsubara
    windows (a few 1e-4)."""
    g = O.Grid(201, 40.0, 2.0)
    q = O.Quad(801, 1, 0.0, 1.0)
    sk = O.sde(O.bare(g, U), O.Prop(D, T), q, q)
    e, imS = g.nodes(), sk[:, 1].imag
    N = 4
    s_mf = MF.sde(MF.bare(MF.MGrid(210, N, T), U), MF.MProp(D, T), 200, 200)
    v = MF.nu(np.arange(-N, N), T)
    spec = np.array([np.trapezoid(-imS / np.pi / (1j * vv - e), e) for vv in v])
    assert np.abs(s_mf - spec).max() < 2e-3 * np.abs(spec).max()
    assert np.abs(s_mf.real).max() < 1e-14  # particle-hole symmetry: Sigma(i nu) imaginary


def test_matsubara_parquet_solution_third_order_expansion():
    """The converged Matsubara parquet state, expanded in U, starts with the second- and
    third-order diagrams: gamma_r = gamma_r^(2) + gamma_r^(3) + O(U^4) with gamma_r^(3) =
    1/2 [B_r(Gamma_0, Gamma^(2)) + B_r(I_r^(2), Gamma_0) + B_r(Gamma_0, I_r^(2)) + B_r(Gamma^(2),
    Gamma_0)] and Sigma = Sigma^(2) + Sigma^(3) + O(U^4) with Sigma^(3) = -1/2 L(B_a(Gamma_0,
    Gamma^(2)), G): the remainders relative to the third-order terms shrink linearly with U."""
    g = MF.MGrid(12, 4, T)
    Nq, Nl = 12, 8
    P0 = MF.MProp(D, T)
    errs = []
    for u in (0.1, 0.05):
        chans, sig, res = MF.parquet_solve(g, u, D, Nq, Nl, alpha=1.0, iterations=40, tol=1e-14)
        assert res[-1] < 1e-13
        g0 = MF.bare(g, u)
        k1 = [MF.bubble(r, g0, g0, P0, Nq).K1 for r in range(3)]
        all2 = MF.MVertex(g, 0.0, [MF.MChannel(1.0, k1[r]) for r in range(3)])
        e_g = 0.0
        for r in range(3):
            i2 = MF.MVertex(g, 0.0, [MF.MChannel(1.0, k1[rr]) if rr != r else MF.MChannel(0.0) for rr in range(3)])
            terms = [MF.bubble(r, g0, all2, P0, Nq), MF.bubble(r, i2, g0, P0, Nq), MF.bubble(r, g0, i2, P0, Nq),
                     MF.bubble(r, all2, g0, P0, Nq)]
            for c in ("K1", "K2", "K2p"):
                third = 0.5 * sum(getattr(t_, c) for t_ in terms)
                second = k1[r] if c == "K1" else 0.0
                e_g = max(e_g, np.abs(getattr(chans[r], c) - second - third).max() / np.abs(third).max())
        s2 = MF.sde(g0, P0, Nq, Nl)
        phi = MF.bubble(0, g0, all2, P0, Nq)
        pv = MF.MVertex(g, 0.0, [MF.MChannel(1.0, phi.K1, None, phi.K2p, None), MF.MChannel(0.0), MF.MChannel(0.0)])
        s3 = -0.5 * MF.loop(pv, P0, Nl)
        e_s = np.abs(sig - s2 - s3).max() / np.abs(s3).max()
        errs.append((e_g, e_s))
    (g1, s1), (g2, s2_) = errs
    assert g1 < 0.2 and s1 < 0.2
    assert 0.3 < g2 / g1 < 0.7 and 0.3 < s2_ / s1 < 0.7


# ---------------------------------------------------------------- Matsubara flow
def test_matsubara_single_scale_lines_are_derivatives():
    """S = dG/dDelta at fixed Sigma and G Sigma_dot G = dG/dh along Sigma + h Sigma_dot (central
    differences); the Pi_dot bubble and the loop with S are the Delta-derivatives of the bubble
    and of the loop at fixed vertex and Sigma."""
    sig = 0.1 * np.exp(1j * np.linspace(0, 2, 12)) - 0.05j
    dsig = 0.2 * np.exp(-1j * np.linspace(0, 1, 12))
    n = np.arange(-9, 9)
    h = 1e-6
    P = MF.MProp(1.3, T, sig)
    fd = (MF.MProp(1.3 + h, T, sig)(n) - MF.MProp(1.3 - h, T, sig)(n)) / (2 * h)
    assert np.abs(P.line(n, 1) - fd).max() < 1e-8 * np.abs(fd).max()
    fd2 = (MF.MProp(1.3, T, sig + h * dsig)(n) - MF.MProp(1.3, T, sig - h * dsig)(n)) / (2 * h)
    assert np.abs(MF.MProp(1.3, T, sig, dsig).line(n, 2) - fd2).max() < 1e-8 * np.abs(fd2).max()
    g = MF.MGrid(3, 3, T)
    V = _random_vertex(g, 5)
    for r in range(3):
        b = MF.bubble(r, V, V, P, 6, 1)
        bp = MF.bubble(r, V, V, MF.MProp(1.3 + h, T, sig), 6)
        bm = MF.bubble(r, V, V, MF.MProp(1.3 - h, T, sig), 6)
        for c in MF.CLASSES:
            d = (getattr(bp, c) - getattr(bm, c)) / (2 * h)
            assert np.abs(getattr(b, c) - d).max() < 1e-7 * np.abs(d).max(), (r, c)
    lp = MF.loop(V, MF.MProp(1.3 + h, T, sig), 7)
    lm = MF.loop(V, MF.MProp(1.3 - h, T, sig), 7)
    d = (lp - lm) / (2 * h)
    assert np.abs(MF.loop(V, P, 7, 1) - d).max() < 1e-7 * np.abs(d).max()


def test_matsubara_flow_of_pt2_reaches_pt2_to_second_order():
    """The one-loop flow of the PT2 state from Delta = 2 to 1 reproduces the PT2 vertex at
    Delta = 1 up to O(U^3) and the Runge-Kutta error: the relative deviation falls linearly
    with U."""
    g = MF.MGrid(12, 4, T)
    Nq, Nl = 12, 8
    devs = []
    for u in (0.1, 0.05):
        chans, sig = MF.pt2_state(g, u, 2.0, Nq, Nl)
        ch, _ = MF.mfrg_flow(g, u, 2.0, 1.0, 4, 1, Nq, Nl, chans, sig)
        ref, _ = MF.pt2_state(g, u, 1.0, Nq, Nl)
        devs.append(max(np.abs(ch[r].K1 - ref[r].K1).max() / np.abs(ref[r].K1).max() for r in range(3)))
    assert devs[0] < 0.05
    assert 0.3 < devs[1] / devs[0] < 0.7


def test_analytic_tails_make_the_bubble_independent_of_the_window():
    """With the analytic tails the summands beyond the window enter through the bare bubble's
    closed form and the vertices' large-frequency values: for Gamma_0 on both sides the K1 class
    is the same for every window (and differs by the window's tail without them), and for random
    vertices with a self-energy on a box the bubble no longer depends on the window once the
    window covers every box (the tails are then exact) -- without them it changes by ten per cent."""
    g = MF.MGrid(6, 4, T)
    g0 = MF.bare(g, U)
    P = MF.MProp(D, T)
    for r in range(3):
        a = MF.bubble(r, g0, g0, P, 5, tails=True).K1
        b = MF.bubble(r, g0, g0, P, 60, tails=True).K1
        c = MF.bubble(r, g0, g0, P, 60).K1
        assert np.abs(a - b).max() < 1e-14 * np.abs(b).max()
        assert np.abs(b - c).max() > 1e-2 * np.abs(b).max()
    g = MF.MGrid(3, 3, T)
    L, R = _random_vertex(g, 1), _random_vertex(g, 2)
    Pd = MF.MProp(D, T, 0.2 * np.exp(1j * np.linspace(0, 3, 10)) - 0.1j)
    for r in range(3):
        ref = MF.bubble(r, L, R, Pd, 40, tails=True)
        for Nq in (8, 20):
            with_t = MF.bubble(r, L, R, Pd, Nq, tails=True)
            without = MF.bubble(r, L, R, Pd, Nq)
            for x in MF.CLASSES:
                scale = np.abs(getattr(ref, x)).max()
                assert np.abs(getattr(with_t, x) - getattr(ref, x)).max() < 1e-13 * scale, (r, Nq, x)
            assert max(np.abs(getattr(without, x) - getattr(ref, x)).max() / np.abs(getattr(ref, x)).max()
                       for x in MF.CLASSES) > 0.05


def test_matsubara_chi_factorises_for_the_bare_vertex_and_diagonalises_the_bubble():
    """With Gamma = Gamma_0 the double sum factorises, chi_r^c = S_r + S_r Gamma_0^c S_r with
    S_r = chi_r at U = 0 = T sum_k Pi_r, and the one-loop K1 class of the bubble is
    pref_r Gamma_0^c S_r Gamma_0^c (prefactors +1, 1/2, -1) only for the channel's own spin
    combinations; at particle-hole symmetry S_p = -S_a."""
    g = MF.MGrid(4, 3, T)
    P = MF.MProp(D, T)
    g0, zero = MF.bare(g, U), MF.bare(g, 0.0)
    combos = {0: ((1, 0), (1, 2)), 1: ((1, 1), (1, -1)), 2: ((0, 1), (2, 1))}
    pref = (1.0, 0.5, -1.0)
    Ss = {}
    for r in range(3):
        S = MF.chi(r, zero, P, 7)
        assert np.abs(S[0] - S[1]).max() == 0.0
        Ss[r] = S[0]
        ch = MF.chi(r, g0, P, 7)
        K1 = MF.bubble(r, g0, g0, P, 7).K1
        for c, (mx, my) in enumerate(combos[r]):
            G0c = mx * (-U) + my * U
            assert np.abs(ch[c] - (S[0] + S[0] * G0c * S[0])).max() < 1e-14
            assert np.abs((mx * K1[0] + my * K1[1]) - pref[r] * G0c * S[0] * G0c).max() < 1e-14
    assert np.abs(Ss[1] + Ss[0]).max() < 1e-14


def test_matsubara_flow_step_control_converges_onto_the_extrapolated_rk4_flow():
    """Cash-Karp step control on the Matsubara flow (two loops, Katanin): at tight tolerances it
    lands on the Richardson extrapolation of RK4 with 6 and 12 steps (the ODE's solution to
    O(h^5)) well inside RK4's own error; a loose tolerance takes fewer steps; the accepted Delta
    values run from 2 to 1."""
    g = MF.MGrid(4, 2, T)
    Nq, Nl, u = 6, 4, 0.8
    chans, sig = MF.pt2_state(g, u, 2.0, Nq, Nl)
    c6, s6 = MF.mfrg_flow(g, u, 2.0, 1.0, 6, 2, Nq, Nl, chans, sig)
    c12, s12 = MF.mfrg_flow(g, u, 2.0, 1.0, 12, 2, Nq, Nl, chans, sig)
    tight, loose = {}, {}
    ch, sg = MF.mfrg_flow(g, u, 2.0, 1.0, 2, 2, Nq, Nl, chans, sig, adaptive=True, atol=1e-10, rtol=1e-8,
                          info=tight)
    MF.mfrg_flow(g, u, 2.0, 1.0, 2, 2, Nq, Nl, chans, sig, adaptive=True, atol=1e-5, rtol=1e-4, info=loose)
    e_ad = e_rk = 0.0
    for r in range(3):
        for x in ("K1", "K2", "K2p", "K3"):
            a, b6, b12 = getattr(ch[r], x), getattr(c6[r], x), getattr(c12[r], x)
            ext = b12 + (b12 - b6) / 15.0
            scale = np.abs(b12).max()
            assert np.abs(a - ext).max() < 1e-6 * scale, (r, x)
            e_ad = max(e_ad, np.abs(a - ext).max() / scale)
            e_rk = max(e_rk, np.abs(b12 - ext).max() / scale)
    assert e_ad < 0.2 * e_rk
    ext = s12 + (s12 - s6) / 15.0
    assert np.abs(sg - ext).max() < 1e-8 * np.abs(s12).max()
    assert len(loose["lambdas"]) < len(tight["lambdas"])
    for inf in (tight, loose):
        assert abs(inf["lambdas"][0] - 2.0) < 1e-12 and abs(inf["lambdas"][-1] - 1.0) < 1e-12


def test_matsubara_interaction_regulator():
    """Interaction flow (G_0 -> lam G_0): S is dG/dlam at fixed Sigma, the Pi_dot bubble is the
    lam-derivative of the bubble, the PT2 vertex scales exactly as lam^2, and the one-loop flow of
    the PT2 state from lam = 0.5 to 1 reaches the PT2 vertex at lam = 1 up to O(U^3)."""
    g = MF.MGrid(6, 3, T)
    Nq, Nl = 8, 6
    sig = 0.2 * np.exp(1j * np.linspace(0.0, 2.0, 10)) - 0.05j
    P = MF.MProp(1.3, T, sig, reg=1, lam=0.7)
    n, h = np.arange(-8, 8), 1e-5
    d = (MF.MProp(1.3, T, sig, reg=1, lam=0.7 + h)(n) - MF.MProp(1.3, T, sig, reg=1, lam=0.7 - h)(n)) / (2 * h)
    assert np.abs(P.line(n, 1) - d).max() < 1e-8 * np.abs(d).max()
    V = MF.bare(g, 1.0)
    bp = MF.bubble(0, V, V, MF.MProp(1.3, T, sig, reg=1, lam=0.7 + h), Nq)
    bm = MF.bubble(0, V, V, MF.MProp(1.3, T, sig, reg=1, lam=0.7 - h), Nq)
    b1 = MF.bubble(0, V, V, P, Nq, 1)
    dk = (bp.K1 - bm.K1) / (2 * h)
    assert np.abs(b1.K1 - dk).max() < 1e-7 * np.abs(dk).max()
    k_half = MF.pt2_state(g, 1.0, 1.0, Nq, Nl, reg=1, lam=0.5)[0]
    k_one = MF.pt2_state(g, 1.0, 1.0, Nq, Nl, reg=1, lam=1.0)[0]
    for r in range(3):
        assert np.abs(k_half[r].K1 - 0.25 * k_one[r].K1).max() < 1e-14 * np.abs(k_one[r].K1).max()
    devs = []
    for u in (0.2, 0.1):
        chans, s0 = MF.pt2_state(g, u, 1.0, Nq, Nl, reg=1, lam=0.5)
        ch, _ = MF.mfrg_flow(g, u, 0.5, 1.0, 4, 1, Nq, Nl, chans, s0, reg=1, Delta=1.0)
        ref, _ = MF.pt2_state(g, u, 1.0, Nq, Nl, reg=1, lam=1.0)
        devs.append(max(np.abs(ch[r].K1 - ref[r].K1).max() / np.abs(ref[r].K1).max() for r in range(3)))
    assert devs[0] < 0.05
    assert 0.3 < devs[1] / devs[0] < 0.7
