"""Pins of the oracle's algebraic frequency grid (Sec. "Frequency grids": an equidistant
auxiliary variable W mapped by v = A W |W| / sqrt(1 - W^2)), here bounded at |v| <= L.

The oracle inverts the map in closed form; these tests check that inverse against the
forward map solved numerically (brentq), a closed-form point (v = A at W^2 = (sqrt(5) - 1)/2),
the quadratic growth near zero that tells this grid from the tangent grid, linear
interpolation in W through the vertex lookup, and that a bubble's outputs sit at the grid's
nodes (the bare bubble at a node equals the bare bubble at that frequency on another grid).
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import oracle as O


def _forward(W, A):
    return A * W * abs(W) / np.sqrt(1.0 - W * W)


def _aux(v, A):
    """W of v by bisection-type root finding on the forward map."""
    if v == 0.0:
        return 0.0
    return brentq(lambda W: _forward(W, A) - v, -1 + 1e-15, 1 - 1e-15, xtol=1e-16, rtol=1e-15)


def _locate_x(g, v):
    i0, t = O.C.c_int(), O.C.c_double()
    assert O.lib().oracle_grid_locate(g.n, g.L, g.a, g.map, v, O.C.byref(i0), O.C.byref(t)) == 1
    return -1.0 + 2.0 * (i0.value + t.value) / (g.n - 1)


@pytest.mark.parametrize("n,L,A", [(31, 20.0, 1.0), (201, 20.0, 0.7), (8, 150.0, 3.0)])
def test_algebraic_nodes_span_the_extent_and_are_odd(n, L, A):
    g = O.Grid(n, L, A, 1)
    v = g.nodes()
    assert abs(v[0] + L) < 1e-12 * L and abs(v[-1] - L) < 1e-12 * L
    assert np.all(np.diff(v) > 0) and np.array_equal(v, -v[::-1])  # exactly odd
    if n % 2:
        assert v[n // 2] == 0.0
    theta = _aux(L, A)
    x = -1.0 + 2.0 * np.arange(n) / (n - 1)
    W = np.array([_aux(vi, A) for vi in v])
    assert np.abs(W - x * theta).max() < 1e-12


def test_algebraic_grid_grows_quadratically_near_zero():
    """v ~ A W^2 at small W: the first nodes off zero go as k^2 (the tangent grid's go as k)."""
    n = 4001
    va, vt = O.Grid(n, 20.0, 1.0, 1).nodes(), O.Grid(n, 20.0, 1.0, 0).nodes()
    c = n // 2
    for k in (2, 3, 5):
        assert va[c + k] / va[c + 1] == pytest.approx(k * k, rel=1e-4)
        assert vt[c + k] / vt[c + 1] == pytest.approx(k, rel=1e-4)


@pytest.mark.parametrize("A", [1.0, 2.5])
def test_algebraic_locate_inverts_the_map(A):
    g = O.Grid(41, 30.0, A, 1)
    theta = _aux(g.L, A)
    # closed form: v = A where W^4 = 1 - W^2
    assert _locate_x(g, A) * theta == pytest.approx(np.sqrt((np.sqrt(5.0) - 1.0) / 2.0), abs=1e-13)
    rng = np.random.default_rng(5)
    for v in np.concatenate([rng.uniform(-g.L, g.L, 40), [1e-9, -3e-4, g.L, -g.L]]):
        assert _locate_x(g, v) * theta == pytest.approx(_aux(v, A), abs=2e-13)
    i0, t = O.C.c_int(), O.C.c_double()
    assert O.lib().oracle_grid_locate(g.n, g.L, g.a, g.map, g.L * 1.01, O.C.byref(i0), O.C.byref(t)) == 0


def test_vertex_lookup_interpolates_linearly_in_the_auxiliary_variable():
    """A K1 class holding x_i (linear in W) reads back W(w)/theta at any w in [-L, L]."""
    g = O.Grid(25, 20.0, 1.3, 1)
    x = -1.0 + 2.0 * np.arange(g.n) / (g.n - 1)
    K1 = np.zeros((2, g.n, 16), complex)
    K1[0] = x[:, None]
    K1[1] = 2.0 * x[:, None]
    V = O.Vertex(g, r0=0.0, ch=[O.Channel(1.0, K1), O.Channel(0.0), O.Channel(0.0)])
    theta = _aux(g.L, g.a)
    ws = np.array([-19.3, -4.2, -0.31, 0.0, 0.05, 1.7, 11.0, 20.0])
    out = O.vertex_eval(V, 0, np.stack([ws, 0 * ws, 0 * ws], 1), parts=O.P_K1)
    ref = np.array([_aux(w, g.a) / theta for w in ws])
    assert np.abs(out[:, 0, :] - ref[:, None]).max() < 1e-12
    assert np.abs(out[:, 1, :] - 2 * ref[:, None]).max() < 1e-12


def test_bubble_outputs_sit_at_the_algebraic_nodes():
    """The bare bubble needs no interpolation, so K1 at node i of the algebraic grid equals K1
    at the end node of a tangent grid whose extent is that node's frequency."""
    P, q = O.Prop(Delta=1.0, T=0.1), O.Quad(301)
    g = O.Grid(15, 20.0, 1.0, 1)
    v = g.nodes()
    for r in range(3):
        k1 = O.bubble(r, O.bare(g, 1.0), O.bare(g, 1.0), P, q, cmask=O.C_K1).K1
        for i in (9, 12, 14):
            gt = O.Grid(3, float(v[i]), 1.0, 0)
            ref = O.bubble(r, O.bare(gt, 1.0), O.bare(gt, 1.0), P, q, cmask=O.C_K1).K1
            assert np.abs(k1[:, i] - ref[:, 2]).max() < 1e-13 * np.abs(ref).max()
