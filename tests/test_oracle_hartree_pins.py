"""Pins of the oracle's Hartree term (Sec. Hartree-Fock, Eq. Hartree): the occupation of a
Lorentzian level against its closed form at finite temperature (digamma function), the
self-consistent term at particle-hole symmetry, the Friedel sum rule as T -> 0, and the
one-shot term with a dynamic self-energy against an independent adaptive integration, and
the asymmetric parquet solver at eps_d = -U/2 reproducing the particle-hole symmetric one.
The asymmetric mfRG flow: the asymptotic value of the loop (Gamma_0 and the t-channel classes
read at zero transfer frequency), its first-order flow as the Hartree term's, and the flow at
eps_d = -U/2 reproducing the symmetric one."""
import numpy as np
import scipy.integrate as si
import scipy.special as sp

import oracle as O

D = 1.0
Q = O.Quad(4001, 1, 0.0, 1.0)


def _n_closed(E, T, Dl=D):
    """int dv n_F(v) (Dl/pi)/((v - E)^2 + Dl^2) = 1/2 - Im psi(1/2 + (Dl + iE)/(2 pi T)) / pi."""
    return 0.5 - sp.psi(0.5 + (Dl + 1j * E) / (2 * np.pi * T)).imag / np.pi


def test_occupation_of_lorentzian_level_matches_closed_form():
    for T in (0.05, 0.1, 0.5):
        for E in (-1.3, -0.2, 0.0, 0.45, 3.0):
            assert abs(O.occupation(E, D, T, Q) - _n_closed(E, T)) < 1e-12


def test_self_consistent_hartree_term_at_particle_hole_symmetry():
    for U in (0.5, 2.0, 4.0):
        sH, it = O.hartree(U, -U / 2, D, 0.1, Q, tol=1e-13)
        assert abs(sH - U / 2) < 1e-12 and it > 10


def test_self_consistent_hartree_term_solves_its_equation_and_friedel_rule():
    """Away from half filling: Sigma_H = U n(eps_d + Sigma_H) to the bracket width; at low T the
    occupation obeys the Friedel sum rule n = 1/2 - arctan((eps_d + Sigma_H)/Delta)/pi."""
    for U, eps_d in ((1.0, -0.2), (2.0, -0.4), (3.0, 0.3)):
        sH, _ = O.hartree(U, eps_d, D, 0.1, Q, tol=1e-13)
        assert abs(sH - U * _n_closed(eps_d + sH, 0.1)) < 1e-11
        sH0, _ = O.hartree(U, eps_d, D, 0.005, O.Quad(8001, 1, 0.0, 0.2), tol=1e-13)
        n = sH0 / U
        assert abs(n - (0.5 - np.arctan((eps_d + sH0) / D) / np.pi)) < 1e-4
        assert 0.0 < n < 1.0


def test_one_shot_hartree_with_dynamic_self_energy():
    """U n with G^R = 1/(v - E + i Delta - Sigma^R(v)), Sigma^R given on the tangent grid and
    interpolated linearly in the auxiliary variable (zero outside): against scipy's adaptive
    integration of the same integrand, interpolation written out here."""
    g = O.Grid(41)
    v = g.nodes()
    sr = 0.3 * (0.4 * np.sin(v) / (1 + v * v) - 1j / (1 + 0.5 * v * v))
    sig = np.zeros((g.n, 4), complex)
    sig[:, 1], sig[:, 2] = sr, np.conj(sr)
    T, U, eps_d, sH = 0.1, 1.5, -0.3, 0.6
    theta = np.arctan(g.L / g.a)
    xs = np.arctan(v / g.a) / theta

    def sig_at(x):
        if abs(x) > g.L:
            return 0.0
        y = np.arctan(x / g.a) / theta
        return np.interp(y, xs, sr.real) + 1j * np.interp(y, xs, sr.imag)

    E = eps_d + sH
    # <n> = 1/2 + (1/2 pi) int tanh(v/2T) Im G^R (n_F = (1 - tanh)/2 and the sum rule for the 1/2)
    f = lambda x: np.tanh(x / (2 * T)) * (1.0 / (x - E + 1j * D - sig_at(x))).imag / (2 * np.pi)
    pts = [-g.L, -2, -1, 0, 1, 2, g.L]
    n = 0.5 + sum(si.quad(f, a, b, epsabs=1e-13, epsrel=1e-12, limit=400)[0] for a, b in zip(pts[:-1], pts[1:]))
    n += si.quad(f, -np.inf, -g.L, epsabs=1e-14, limit=200)[0] + si.quad(f, g.L, np.inf, epsabs=1e-14, limit=200)[0]
    got, _ = O.hartree(U, eps_d, D, T, O.Quad(20001, 1, 0.0, 1.0), g, sig, self_consistent=False, sigma_H=sH)
    assert abs(got - U * n) < 1e-6 * U


def test_asymmetric_parquet_solver_at_half_filling_is_the_symmetric_one():
    g, q = O.Grid(9), O.Quad(31)
    U = 1.0
    c0, s0, r0 = O.parquet_solve(g, U, D, 0.1, q, q, iterations=4)
    c1, s1, r1, sH = O.parquet_solve(g, U, D, 0.1, q, q, iterations=4, eps_d=-U / 2, q_hartree=Q, hartree_tol=1e-14)
    assert abs(sH - U / 2) < 1e-13
    assert np.allclose(r0, r1, rtol=1e-10, atol=0)
    for r in range(3):
        for x in O.CLASSES:
            a, b = getattr(c0[r], x), getattr(c1[r], x)
            assert np.abs(a - b).max() <= 1e-12 * max(np.abs(a).max(), 1e-300)
    assert np.abs(s1 - s0).max() < 1e-12 * np.abs(s0).max()


def test_asymmetric_parquet_solver_contracts_with_the_hartree_entry():
    """Away from half filling the Hartree term stays within (0, U) (occupation within (0, 1)) and
    the solver with the Hartree entry in its state contracts."""
    g, q = O.Grid(9), O.Quad(31)
    U, eps_d = 1.0, -0.2
    _, _, res, sH = O.parquet_solve(g, U, D, 0.1, q, q, iterations=6, eps_d=eps_d, q_hartree=Q)
    assert 0.0 < sH < U and res[-1] < 0.15 * res[0]
    assert res[-1] < res[-2] < res[-3]


# ---------------------------------------------------------------- asymmetric mfRG flow
def _zero_state(n):
    z = lambda sh: np.zeros(sh, complex)
    return [O.Channel(1.0, z((2, n, 16)), z((2, n, n, 16)), z((2, n, n, 16)), z((2, n, n, n, 16))) for _ in range(3)]


def test_static_part_of_the_loop_is_the_same_at_every_frequency():
    """In the loop's legs (v, v_j | v, v_j) the t channel sits at transfer frequency 0 with first
    fermionic frequency v_j: a vertex made of Gamma_0, K1_t and K2_t gives the same loop at every
    grid frequency -- the asymptotic value the flow of the asymmetric model carries beyond the
    grid -- and loop_static is that value for any vertex; adding K2'_t (read at v) breaks it."""
    from workload import random_channel
    n = 9
    g, q, P = O.Grid(n), O.Quad(31), O.Prop(D, 0.1, eps=0.3)
    c = random_channel(n, 7, 0.3)
    Vs = O.Vertex(g, 1.0, [O.Channel(0.0), O.Channel(0.0), O.Channel(0.8, c["K1"], c["K2"], None, None)])
    L = O.loop(Vs, P, q)
    assert np.abs(L - L[0]).max() < 1e-13 * np.abs(L).max()
    full = [random_channel(n, s_, 0.3) for s_ in (1, 2)]
    V = O.Vertex(g, 1.0, [O.Channel(1.0, *[f[x] for x in O.CLASSES]) for f in full]
                 + [O.Channel(0.8, c["K1"], c["K2"], c["K2p"], c["K3"])])
    assert np.abs(O.loop_static(V, P, q) - L[0]).max() < 1e-14 * np.abs(L).max()
    Vp = O.Vertex(g, 1.0, [O.Channel(0.0), O.Channel(0.0), O.Channel(0.8, c["K1"], c["K2"], c["K2p"], None)])
    Lp = O.loop(Vp, P, q)
    assert np.abs(Lp - Lp[0]).max() > 1e-3 * np.abs(Lp).max()


def test_asymmetric_flow_of_the_asymptotic_value_is_the_hartree_flow_at_first_order():
    """Flowing the bare state (Gamma = Gamma_0, Sigma = 0) of the level eps_d from Delta = 2 to 1,
    the self-energy beyond the grid changes by U [<n>(Delta = 1) - <n>(Delta = 2)] + O(U^2),
    <n> the occupation of the bare level (pinned above against its closed form): the first-order
    flow -L(Gamma_0, S) is the Delta-derivative of the Hartree term.  The relative deviation
    halves with U."""
    n = 9
    g, qb, ql = O.Grid(n), O.Quad(31), O.Quad(401, 1, 0.0, 1.0)
    T, ed = 0.1, 0.4
    devs = []
    for U in (0.1, 0.05):
        _, _, info = O.mfrg_flow(g, U, T, 2.0, 1.0, 4, 1, qb, ql, _zero_state(n), np.zeros((n, 4), complex),
                                 O.FlowOptions(), eps_d=ed, sigma_inf=0.0)
        ref = U * (O.occupation(ed, 1.0, T, Q) - O.occupation(ed, 2.0, T, Q))
        assert abs(ref) > 1e-3 * U
        devs.append(abs(info["sigma_inf"] - ref) / abs(ref))
    assert devs[0] < 0.03 and 0.4 < devs[1] / devs[0] < 0.6


def test_asymmetric_flow_at_half_filling_is_the_symmetric_flow():
    """At eps_d = -U/2 with the Hartree value U/2 as the initial self-energy beyond the grid, the
    asymmetric flow (level eps_d + Sigma_inf, Sigma_inf flowing with the asymptotic value of the
    loops) is the symmetric flow: Sigma_inf stays U/2 (the static part of Sigma vanishes at
    particle-hole symmetry) and the channels and the rest of Sigma agree to rounding; multiloop
    order 3, Katanin, self-energy corrections."""
    n, U, T = 9, 1.0, 0.1
    g, q = O.Grid(n), O.Quad(31)
    chans, sig = O.pt2_state(g, U, 2.0, T, q, q)
    fo = O.FlowOptions(se_iterations=3)
    c1, s1, _ = O.mfrg_flow(g, U, T, 2.0, 1.0, 2, 3, q, q, chans, sig, fo)
    c2, s2, info = O.mfrg_flow(g, U, T, 2.0, 1.0, 2, 3, q, q, chans, sig, fo, eps_d=-U / 2, sigma_inf=U / 2)
    assert abs(info["sigma_inf"] - U / 2) < 1e-14
    assert np.abs(s2 - s1).max() < 1e-13 * np.abs(s1).max()
    for r in range(3):
        for x in O.CLASSES:
            a, b = getattr(c2[r], x), getattr(c1[r], x)
            assert np.abs(a - b).max() <= 1e-13 * max(np.abs(b).max(), 1e-300), (r, x)
