"""Pins of the oracle's adaptive Gauss-Lobatto-Kronrod integration (Sec. Frequency integration):
the three rules against the node values the paper prints and against their degrees of
exactness, the adaptive integrator on integrals with closed forms (a narrow Lorentzian, a kink),
the per-node bubble integrand against the pinned fixed-quadrature bubble, and the adaptive
bubble against the fixed-quadrature bubble as its node count grows."""
import os

import numpy as np

import oracle as O
from workload import random_channel

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", "glk_nodes.txt")) if ln.strip() and ln[0] != "#"]
    return {k: [float(v) for kk, v in rows if kk == k] for k in ("gl4", "glk7", "glk13")}


def test_rule_nodes_match_the_printed_distribution():
    (x7, w4), (_, w7), (x13, w13) = O.glk_rules()
    gold = _golden()
    pos7, pos13 = set(np.round(x7[x7 >= 0], 6)), np.round(x13[x13 >= 0], 6)
    gl4 = np.round(x7[(w4 > 0) & (x7 >= 0)], 6)
    assert sorted(gl4) == sorted(np.round(gold["gl4"], 6))
    assert set(np.round(gold["glk7"], 6)) <= pos7 and set(np.round(gold["gl4"], 6)) <= pos7
    new13 = sorted(set(pos13) - pos7)
    assert np.allclose(new13, sorted(gold["glk13"]), atol=6e-7)
    assert abs(x7[-2] - np.sqrt(2 / 3)) < 1e-15 and abs(x7[-3] - 1 / np.sqrt(5)) < 1e-15


def test_rule_degrees_of_exactness():
    (x7, w4), (_, w7), (x13, w13) = O.glk_rules()
    for x, w, deg in ((x7, w4, 5), (x7, w7, 9), (x13, w13, 18)):
        for k in range(deg + 1):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs(w @ x ** k - exact) < 1e-14
        k = deg + 1 if (deg + 1) % 2 == 0 else deg + 2
        assert abs(w @ x ** k - 2.0 / (k + 1)) > 1e-7


def test_adaptive_integrator_on_closed_forms():
    # narrow Lorentzian and a kink; vector-valued (two components at once)
    f = lambda x: np.stack([1.0 / (x * x + 1e-4), np.abs(x - 0.3) + np.cos(3 * x)], axis=1)
    exact = np.array([2 / 0.01 * np.arctan(100.0), 0.5 * 1.3 ** 2 + 0.5 * 0.7 ** 2 + 2 * np.sin(3.0) / 3])
    errs, counts = [], []
    for eps in (1e-6, 1e-10):
        val, c = O.adaptive_glk(f, -1.0, 1.0, eps)
        errs.append(np.abs(val - exact).max() / np.abs(exact).max())
        counts.append(c)
    assert errs[0] < 1e-5 and errs[1] < 1e-9 and counts[1] > counts[0] > 1
    # a polynomial of degree 5 is integrated exactly by GL4 and GLK7 and accepted at once
    val, c = O.adaptive_glk(lambda x: (x ** 5 + 3 * x ** 4 + 1.0)[:, None], -1.0, 1.0, 1e-12)
    assert c == 1 and abs(val[0] - (6 / 5 + 2)) < 1e-14
    # an integral that vanishes falls back to the integrand's size for its scale and terminates
    val, c = O.adaptive_glk(lambda x: (x ** 3)[:, None], -1.0, 1.0, 1e-12)
    assert c == 1 and abs(val[0]) < 1e-15


def _vertex(n, seeds=(3, 4, 5), amp=0.3):
    chans = [random_channel(n, s, amp) for s in seeds]
    return O.Vertex(O.Grid(n), 0.8, [O.Channel(1.0, *[c[x] for x in O.CLASSES]) for c in chans])


def _pts(n):
    return np.array([[1, 1, 0, 0], [2, 2, 1, 0], [4, 0, 0, 3], [8, 1, 2, 3], [8, n - 1, 0, n - 1]])


def test_integrand_reproduces_the_fixed_quadrature_bubble():
    n = 5
    V = _vertex(n)
    P = O.Prop(1.0, 0.1)
    q = O.Quad(41)
    v, w = q.nodes_weights()
    for r in range(3):
        ref = O.bubble_points(r, V, V, P, q, _pts(n))
        s = np.tensordot(w, O.bubble_integrand(r, V, V, P, _pts(n), v), axes=([0], [1]))
        assert np.abs(s - ref).max() < 1e-13 * np.abs(ref).max()


def test_adaptive_bubble_is_the_limit_of_the_fixed_quadrature():
    n = 5
    V = _vertex(n)
    P = O.Prop(1.0, 0.1)
    for r in range(3):
        ada, counts = O.bubble_adaptive_points(r, V, V, P, O.Quad(1), _pts(n), 1e-10)
        d = [np.abs(O.bubble_points(r, V, V, P, O.Quad(nq), _pts(n)) - ada).max() / np.abs(ada).max()
             for nq in (401, 1601)]
        # the vertex interpolation has kinks, so the fixed rule converges onto the adaptive value
        # at about h^2: four times the nodes, at most a third of the deviation
        assert d[1] < 1e-4 and d[0] / d[1] > 3.0, (r, d)
        assert min(counts) > 1
