"""Pins of the oracle's fixed-point solver (Sec. parquet solver: mixing, automatic reduction of
the mixing factor, Anderson acceleration) against properties the mathematics fixes: Anderson
acceleration with a full history solves a linear fixed-point problem of real dimension d in
d + 1 updates (its equivalence with GMRES), even where plain iteration diverges; depth 0 is
linear mixing; halving the mixing factor on a growing residual rescues an oscillating map;
on the parquet equations Anderson reaches a smaller residual than linear mixing.  And the three
forms of the Schwinger-Dyson equation combined by the solver: the t-form equals the a-form for
crossing-symmetric vertices, all agree at second order, and their mean has no third-order part
at particle-hole symmetry, where the exact self-energy is even in U."""
import numpy as np

import oracle as O


def _linear_problem(n=3, radius=1.5, seed=1):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    A *= radius / np.abs(np.linalg.eigvals(A)).max()
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    return A, b, np.linalg.solve(np.eye(n) - A, b)


def _maxres(x, g):
    return float(np.abs(g - x).max())


def test_anderson_with_full_history_solves_linear_problem_in_d_plus_one_updates():
    A, b, xs = _linear_problem()
    F = lambda x: A @ x + b
    x, res, _ = O.fixed_point_solve(F, np.zeros(3, complex), _maxres, alpha=1.0, depth=6, iterations=8)
    assert np.abs(x - xs).max() < 1e-12 * np.abs(xs).max()
    assert res[7] < 1e-10 * res[0]
    # plain iteration diverges on this map (spectral radius 1.5), short histories do not solve it
    x0, res0, _ = O.fixed_point_solve(F, np.zeros(3, complex), _maxres, alpha=1.0, depth=0, iterations=8)
    assert res0[-1] > res0[0]
    x2, _, _ = O.fixed_point_solve(F, np.zeros(3, complex), _maxres, alpha=1.0, depth=2, iterations=8)
    assert np.abs(x2 - xs).max() > 1e-3


def test_depth_zero_is_linear_mixing():
    A, b, xs = _linear_problem(radius=0.6, seed=2)
    F = lambda x: A @ x + b
    x, res, _ = O.fixed_point_solve(F, np.zeros(3, complex), _maxres, alpha=0.4, depth=0, iterations=7)
    y = np.zeros(3, complex)
    for _ in range(7):
        y = y + 0.4 * (F(y) - y)
    assert np.abs(x - y).max() < 1e-15


def test_reducing_alpha_rescues_an_oscillating_map():
    """x = -1.5 x + 1 (fixed point 0.4): alpha = 1 oscillates with growing amplitude; halving
    alpha on every growing residual reaches alpha = 0.5 (contraction factor 0.25)."""
    F = lambda x: -1.5 * x + 1.0
    x0 = np.array([0.0 + 0.0j])
    xd, resd, _ = O.fixed_point_solve(F, x0, _maxres, alpha=1.0, iterations=12)
    assert resd[-1] > resd[0]
    x, res, a = O.fixed_point_solve(F, x0, _maxres, alpha=1.0, iterations=40, tol=1e-13, reduce_alpha=True)
    assert a == 0.5 and abs(x[0] - 0.4) < 1e-12


def test_anderson_accelerates_the_parquet_solver():
    g, q = O.Grid(11, 10.0, 1.0), O.Quad(61, 0, 10.0, 1.0)
    _, _, lin = O.parquet_solve(g, 1.0, 1.0, 0.1, q, q, alpha=0.5, iterations=8)
    _, _, And = O.parquet_solve(g, 1.0, 1.0, 0.1, q, q, alpha=0.5, iterations=8, depth=3)
    assert lin[:2] == And[:2]  # the first update has no history
    assert And[-1] < 0.2 * lin[-1]


# ---------------------------------------------------------------- crossing of a closed bubble
def _pt2_vertex(n, nq, U=1.0):
    g, q, P = O.Grid(n), O.Quad(nq), O.Prop(1.0, 0.1)
    k1 = O.pt2_k1(g, U, P, q)
    z2, z3 = np.zeros((2, n, n, 16), complex), np.zeros((2, n, n, n, 16), complex)
    return O.Vertex(g, U, [O.Channel(1.0, k1[r], z2, z2, z3) for r in range(3)]), g, q, P


def test_crossed_closure_of_t_bubble_is_the_loop_of_the_mirrored_a_bubble():
    """For a crossing-symmetric vertex (Gamma_0 plus the PT2 channels), the t bubble B_t(Gamma_0,
    Gamma) closed between legs 2' and 1 (summed literally over Keldysh indices and spins) is
    minus the loop of the a bubble B_a(Gamma, Gamma_0), exactly: the crossing 1 <-> 2 maps the
    one onto the other in the discrete scheme (one grid for every channel)."""
    V, g, q, P = _pt2_vertex(9, 31)
    B = O.bare(g, 1.0)
    bt = O.bubble(2, B, V, P, q)
    ct = O.t_closure(O.Vertex(g, 0.0, [O.Channel(0.0), O.Channel(0.0), O.Channel(1.0, bt.K1, bt.K2, bt.K2p, bt.K3)]),
                     P, q)
    bm = O.bubble(0, V, B, P, q)
    lm = O.loop(O.Vertex(g, 0.0, [O.Channel(1.0, bm.K1, bm.K2, bm.K2p, bm.K3), O.Channel(0.0), O.Channel(0.0)]), P, q)
    assert np.abs(ct + lm).max() < 1e-13 * np.abs(ct).max()


# ---------------------------------------------------------------- the three forms of the SDE
def _second_level_vertex(n, nq, U=1.0, Dl=1.0, Tl=0.1):
    """Gamma_0 plus one and two rounds of bubbles in every channel: crossing symmetric."""
    g, q, P = O.Grid(n), O.Quad(nq), O.Prop(Dl, Tl)
    g0 = O.bare(g, U)
    V1 = O.combine(g, [(r, O.bubble(r, g0, g0, P, q), 1.0) for r in range(3)], r0=U)
    V2 = O.combine(g, [(r, O.bubble(r, V1, V1, P, q), 1.0) for r in range(3)], r0=U)
    return g0, V1, V2, g, q, P


def test_t_form_of_the_sde_is_the_a_form_for_crossing_symmetric_vertices():
    """The t-form of the SDE (B_t(Gamma_0, Gamma) closed between its legs 2 and 1', summed
    literally over Keldysh indices and spins) equals the a-form -1/2 L(B_a(Gamma_0, Gamma), G)
    exactly when Gamma is crossing symmetric: the crossing 1' <-> 2' maps the one diagram onto
    the other.  For a vertex without that symmetry the two differ (the identity is not empty)."""
    g0, V1, V2, g, q, P = _second_level_vertex(7, 25)
    for V in (g0, V1, V2):
        a = O.sde(V, P, q, q)
        t = O.sde_t(V, P, q, q)
        assert np.abs(a).max() > 1e-3
        assert np.abs(t - a).max() < 1e-13 * np.abs(a).max()
    from workload import random_channel
    chs = [random_channel(7, s, 0.3) for s in (1, 2, 3)]
    Vr = O.Vertex(g, 1.0, [O.Channel(1.0, c["K1"], c["K2"], c["K2p"], c["K3"]) for c in chs])
    a, t = O.sde(Vr, P, q, q), O.sde_t(Vr, P, q, q)
    assert np.abs(t - a).max() > 0.1 * np.abs(a).max()


def test_three_sde_forms_agree_at_second_order():
    """With Gamma = Gamma_0 the three forms are the second-order self-energy, to rounding."""
    g0, _, _, g, q, P = _second_level_vertex(9, 31)
    a = O.sde(g0, P, q, q)
    for f in (O.sde_p, O.sde_t, O.sde_average):
        assert np.abs(f(g0, P, q, q) - a).max() < 1e-13 * np.abs(a).max()


def test_mean_of_the_sde_forms_has_no_third_order_part_at_particle_hole_symmetry():
    """At particle-hole symmetry the dynamic self-energy is even in U (the particle-hole
    transformation of one spin species maps U to -U and leaves the other spin's propagator
    unchanged), so its third-order part vanishes.  With Gamma = Gamma_0 + sum_r B_r(Gamma_0,
    Gamma_0) (exact to second order) each single form of the SDE has a third-order part of a few
    per cent of the second order on these grids -- the discretisation -- while the mean of the
    three forms has none, to rounding, at every grid, temperature and hybridisation tried.  A
    wrong normalisation or sign of the p-form, or a dropped form, leaves a third-order part."""
    for n, nq, Dl, Tl in ((9, 31, 1.0, 0.1), (13, 41, 0.5, 0.05)):
        g0, V1, _, g, q, P = _second_level_vertex(n, nq, 1.0, Dl, Tl)
        s2 = O.sde(g0, P, q, q)
        scale = np.abs(s2).max()
        a3 = O.sde(V1, P, q, q) - s2
        p3 = O.sde_p(V1, P, q, q) - O.sde_p(g0, P, q, q)
        m3 = O.sde_average(V1, P, q, q) - O.sde_average(g0, P, q, q)
        assert np.abs(a3).max() > 5e-3 * scale and np.abs(p3).max() > 5e-3 * scale
        assert np.abs(m3).max() < 1e-13 * scale


def test_parquet_solution_with_the_mean_sde_deviates_from_pt2_at_fourth_order():
    """The converged parquet self-energy at particle-hole symmetry, Sigma = Sigma^(2) + O(U^4)
    with the mean of the SDE's forms (no third order, as for the exact self-energy), but
    Sigma^(2) + O(U^3) with the a-form alone (its discretised third order): halving U quarters
    the deviation relative to Sigma^(2) in the one case and halves it in the other."""
    g, q = O.Grid(9), O.Quad(31)
    P0 = O.Prop(1.0, 0.1)
    dev = {}
    for forms in (1, 3):
        for u in (0.4, 0.2):
            _, sig, res = O.parquet_solve(g, u, 1.0, 0.1, q, q, alpha=1.0, iterations=60, tol=1e-14,
                                          sde_forms=forms)
            assert res[-1] < 1e-13
            s2 = O.sde(O.bare(g, u), P0, q, q)
            dev[(forms, u)] = np.abs(sig - s2).max() / np.abs(s2).max()
    r1 = dev[(1, 0.4)] / dev[(1, 0.2)]
    r3 = dev[(3, 0.4)] / dev[(3, 0.2)]
    assert 1.6 < r1 < 2.4
    assert 3.5 < r3 < 4.5
