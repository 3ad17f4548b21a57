"""Pins of the oracle's fixed-point solver (Sec. parquet solver: mixing, automatic reduction of
the mixing factor, Anderson acceleration) against properties the mathematics fixes: Anderson
acceleration with a full history solves a linear fixed-point problem of real dimension d in
d + 1 updates (its equivalence with GMRES), even where plain iteration diverges; depth 0 is
linear mixing; halving the mixing factor on a growing residual rescues an oscillating map;
on the parquet equations Anderson reaches a smaller residual than linear mixing."""
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
