"""Pins of the oracle's flow machinery (Sec. mfRG, Sec. ODE solver, Sec. Flow schemes) against
what the mathematics fixes: single-scale propagators as Lambda-derivatives of G for every
regulator, the Katanin and G Sigma_dot G propagators as directional derivatives, the FDR and
causality of every regulated propagator, the exact rescaling of the interaction flow, the
order conditions of the Cash-Karp pair, the Lambda(t) reparametrisation, and the order in U
of the multiloop self-energy corrections."""
import numpy as np
import pytest

import oracle as O
from workload import random_channel

T = 0.1
NU = np.array([-7.3, -2.0, -0.61, -0.05, 0.0, 0.013, 0.4, 1.7, 3.3, 11.0])


def _sigma(grid, amp=0.3, phase=0.0, temp=T):
    """A smooth causal self-energy on the grid obeying the FDR at temperature temp ([n, 4]:
    Sigma^K at 0, Sigma^R at 1)."""
    v = grid.nodes()
    sr = amp * (0.4 * np.sin(v + phase) / (1 + v * v) - 1j / (1 + 0.5 * v * v))
    sig = np.zeros((grid.n, 4), complex)
    sig[:, 1] = sr
    sig[:, 2] = np.conj(sr)
    sig[:, 0] = 2j * np.tanh(v / (2 * temp)) * sr.imag
    return sig


PARAMS = {O.REG_DELTA: 0.8, O.REG_U: 0.7, O.REG_T: 0.3, O.REG_NU: 0.4}


def _prop(reg, lam, grid, sig, dsig=None):
    return O.flow_prop(grid, reg, lam, 1.0, T, sig, dsig)


@pytest.mark.parametrize("reg", [O.REG_DELTA, O.REG_U, O.REG_T, O.REG_NU])
def test_single_scale_propagator_is_the_lambda_derivative(reg):
    """S = dG/dLambda at fixed Sigma (central differences, h = 1e-5), every regulator."""
    g = O.Grid(15)
    sig = _sigma(g)
    lam, h = PARAMS[reg], 1e-5
    S = O.propagator(_prop(reg, lam, g, sig), NU, kind=1)
    fd = (O.propagator(_prop(reg, lam + h, g, sig), NU) - O.propagator(_prop(reg, lam - h, g, sig), NU)) / (2 * h)
    assert np.abs(S - fd).max() < 1e-7 * np.abs(S).max()
    assert np.abs(S).max() > 1e-3


@pytest.mark.parametrize("reg", [O.REG_DELTA, O.REG_U, O.REG_T, O.REG_NU])
def test_katanin_and_sigma_dot_propagators_are_directional_derivatives(reg):
    """S + G Sigma_dot G = d/dh G(Lambda + h, Sigma + h Sigma_dot) and G Sigma_dot G = d/dh G(Lambda,
    Sigma + h Sigma_dot) at h = 0 (Sigma and Sigma_dot on the same grid, interpolated linearly)."""
    g = O.Grid(15)
    sig, dsig = _sigma(g), _sigma(g, 0.7, 1.1)
    lam, h = PARAMS[reg], 1e-5
    kat = O.propagator(_prop(reg, lam, g, sig, dsig), NU, kind=1)
    fd = (O.propagator(_prop(reg, lam + h, g, sig + h * dsig), NU)
          - O.propagator(_prop(reg, lam - h, g, sig - h * dsig), NU)) / (2 * h)
    assert np.abs(kat - fd).max() < 1e-7 * np.abs(kat).max()
    gsg = O.propagator(_prop(reg, lam, g, sig, dsig), NU, kind=2)
    fd = (O.propagator(_prop(reg, lam, g, sig + h * dsig), NU) - O.propagator(_prop(reg, lam, g, sig - h * dsig), NU)) / (2 * h)
    assert np.abs(gsg - fd).max() < 1e-7 * np.abs(gsg).max()
    assert np.abs(gsg).max() > 1e-3


@pytest.mark.parametrize("reg", [O.REG_DELTA, O.REG_U, O.REG_T, O.REG_NU])
def test_regulated_propagators_obey_fdr_and_causality(reg):
    """With Sigma in equilibrium, G^K = (G^R - G^A) tanh(v/2T) and Im G^R <= 0 (with a dynamic
    Sigma at its grid nodes, where the linear interpolation of Sigma^K is exact)."""
    g = O.Grid(15)
    temp = PARAMS[reg] if reg == O.REG_T else T
    for sig, nu in ((None, NU), (_sigma(g, temp=temp), g.nodes())):
        P = _prop(reg, PARAMS[reg], g, sig)
        m = O.propagator(P, nu)
        GR, GA, GK = m[:, 1, 0], m[:, 0, 1], m[:, 1, 1]
        t = P.T
        assert np.abs(GK - (GR - GA) * np.tanh(nu / (2 * t))).max() < 1e-13 * np.abs(GK).max()
        assert np.all(GR.imag <= 1e-15)
        assert np.abs(GA - np.conj(GR)).max() == 0.0 and np.abs(m[:, 0, 0]).max() == 0.0


def test_regulators_reduce_to_the_physical_propagator():
    """Interaction flow at Lambda = 1 gives the unregulated G; the frequency flow approaches it
    as Lambda -> 0 at every v != 0 (linearly in Lambda / |v|)."""
    g = O.Grid(15)
    sig = _sigma(g)
    nu = NU[NU != 0.0]
    ref = O.propagator(O.sigma_prop(g, 1.0, T, sig), nu)
    m = O.propagator(O.flow_prop(g, O.REG_U, 1.0, 1.0, T, sig), nu)
    assert np.abs(m - ref).max() < 1e-14 * np.abs(ref).max()
    d = [np.abs(O.propagator(O.flow_prop(g, O.REG_NU, lam, 1.0, T, sig), nu) - ref).max() for lam in (1e-6, 1e-7)]
    assert d[0] < 1e-3 and 8 < d[0] / d[1] < 12


def test_interaction_flow_rescales_exactly():
    """G_0 -> Lambda G_0 is U -> Lambda^2 U with Sigma -> Sigma / Lambda and Gamma -> Gamma /
    Lambda^2 (Sec. U-flow): PT2 K1 and Sigma^(2) at Lambda equal the unregulated ones at
    Lambda^2 U, rescaled, in the discrete scheme as well."""
    g, q = O.Grid(11), O.Quad(41)
    U, lam = 0.9, 0.6
    P = O.flow_prop(g, O.REG_U, lam, 1.0, T, None)
    k1 = O.pt2_k1(g, U, P, q)
    k1r = O.pt2_k1(g, lam * lam * U, O.Prop(1.0, T), q)
    for r in range(3):
        assert np.abs(k1[r] - k1r[r] / lam ** 2).max() < 1e-13 * np.abs(k1[r]).max()
    s = O.sde(O.bare(g, U), P, q, q)
    sr = O.sde(O.bare(g, lam * lam * U), O.Prop(1.0, T), q, q)
    assert np.abs(s - sr / lam).max() < 1e-13 * np.abs(s).max()


def test_katanin_bubble_is_the_derivative_of_the_bubble():
    """B_r(Gamma, Gamma; Pidot) with the Katanin propagator is d/dh B_r(Gamma, Gamma; Pi[G(Lambda + h,
    Sigma + h Sigma_dot)]) (central differences), every channel."""
    n, nq = 7, 21
    g, q = O.Grid(n), O.Quad(nq)
    chans = [random_channel(n, s, 0.3) for s in (3, 4, 5)]
    V = O.Vertex(g, 0.8, [O.Channel(1.0, *[c[x] for x in O.CLASSES]) for c in chans])
    sig, dsig = _sigma(g), _sigma(g, 0.7, 1.1)
    lam, h = 1.3, 1e-5
    for r in range(3):
        ref = O.bubble(r, V, V, O.flow_prop(g, O.REG_DELTA, lam, 1.0, T, sig, dsig), q, 1)
        bp = O.bubble(r, V, V, O.flow_prop(g, O.REG_DELTA, lam + h, 1.0, T, sig + h * dsig), q)
        bm = O.bubble(r, V, V, O.flow_prop(g, O.REG_DELTA, lam - h, 1.0, T, sig - h * dsig), q)
        for c in O.CLASSES:
            a, fd = getattr(ref, c), (getattr(bp, c) - getattr(bm, c)) / (2 * h)
            assert np.abs(a - fd).max() < 1e-7 * np.abs(a).max(), (r, c)


def test_loop_with_sigma_dot_is_the_derivative_of_the_loop():
    """L(Gamma, G Sigma_dot G) = d/dh L(Gamma, G[Sigma + h Sigma_dot])."""
    n, nq = 9, 31
    g, q = O.Grid(n), O.Quad(nq)
    chans = [random_channel(n, s, 0.3) for s in (6, 7, 8)]
    V = O.Vertex(g, 0.8, [O.Channel(1.0, *[c[x] for x in O.CLASSES]) for c in chans])
    sig, dsig = _sigma(g), _sigma(g, 0.7, 1.1)
    h = 1e-5
    a = O.loop(V, O.flow_prop(g, O.REG_DELTA, 1.0, 1.0, T, sig, dsig), q, kind=2)
    fd = (O.loop(V, O.sigma_prop(g, 1.0, T, sig + h * dsig), q) - O.loop(V, O.sigma_prop(g, 1.0, T, sig - h * dsig), q)) / (2 * h)
    assert np.abs(a - fd).max() < 1e-7 * np.abs(a).max()


def test_cash_karp_order_conditions():
    """Row sums of the stage matrix equal the nodes; the fourth-order weights satisfy the eight
    order conditions up to order 4, the fifth-order weights also the order-5 quadrature and
    tall-tree conditions, and the fourth-order weights fail the order-5 quadrature condition."""
    c = np.array(O.CK_C)
    A = np.zeros((6, 6))
    for i, row in enumerate(O.CK_A):
        A[i, :len(row)] = row
    assert np.allclose(A.sum(1), c, atol=1e-15, rtol=0)
    for b in (np.array(O.CK_B4), np.array(O.CK_B5)):
        conds = [(b.sum(), 1), (b @ c, 1 / 2), (b @ c ** 2, 1 / 3), (b @ (A @ c), 1 / 6), (b @ c ** 3, 1 / 4),
                 (b @ (c * (A @ c)), 1 / 8), (b @ (A @ c ** 2), 1 / 12), (b @ (A @ (A @ c)), 1 / 24)]
        for got, want in conds:
            assert abs(got - want) < 1e-14
    b5, b4 = np.array(O.CK_B5), np.array(O.CK_B4)
    for got, want in ((b5 @ c ** 4, 1 / 5), (b5 @ (A @ (A @ (A @ c))), 1 / 120), (b5 @ (c * c * (A @ c)), 1 / 10)):
        assert abs(got - want) < 1e-14
    assert abs(b4 @ c ** 4 - 1 / 5) > 1e-4


def test_ode_solver_reaches_tolerance_and_lands_on_the_end():
    """y' = -2 t y + cos t on [0, 3] (closed form via the integrating factor is not needed:
    compare with the fixed-step RK4 at 4000 steps); the adaptive error shrinks with the
    tolerance, needs more steps for tighter tolerances, and the last step lands on t1."""
    f = lambda t, y: -2 * t * y + np.cos(t) * np.ones_like(y)
    y0 = np.array([1.0 + 0.5j])
    ref, _, _ = O.ode_solve(f, y0, 0.0, 3.0, 4000)
    errs, nsteps = [], []
    for tol in (1e-4, 1e-7, 1e-10):
        y, ts, rej = O.ode_solve(f, y0, 0.0, 3.0, 4, adaptive=True, atol=tol, rtol=tol, max_steps=10000)
        assert ts[-1] == 3.0
        errs.append(abs(y[0] - ref[0]))
        nsteps.append(len(ts) - 1)
    assert errs[0] < 1e-3 and errs[2] < errs[1] < errs[0] and errs[2] < 1e-8
    assert nsteps[0] < nsteps[1] < nsteps[2]


def test_delta_flow_reparametrisation():
    """Lambda(t) = 5 t|t| / sqrt(1 - t^2): inverse, derivative, oddness, monotonicity."""
    ts = np.linspace(-0.95, 0.95, 39)
    lam = np.array([O.flow_lambda(O.REG_DELTA, t) for t in ts])
    assert np.all(np.diff(lam) > 0)
    back = np.array([O.flow_t(O.REG_DELTA, x) for x in lam])
    assert np.abs(back - ts).max() < 1e-13
    h = 1e-6
    for t in (-0.7, 0.1, 0.4255, 0.9):
        fd = (O.flow_lambda(O.REG_DELTA, t + h) - O.flow_lambda(O.REG_DELTA, t - h)) / (2 * h)
        assert abs(fd - O.flow_dlambda_dt(O.REG_DELTA, t)) < 1e-7 * abs(fd)
    assert O.flow_lambda(O.REG_U, 0.3) == 0.3 and O.flow_t(O.REG_T, 0.3) == 0.3


def test_self_energy_corrections_are_fourth_order_and_converge():
    """The multiloop self-energy corrections start at U^4 (the centre terms of l = 3 are of
    order U^4, the t-term one order higher): the change they make to Sigma_dot falls by 16
    when U halves; below three loops there is none; the iteration converges."""
    n, nq = 9, 31
    g, q = O.Grid(n), O.Quad(nq)
    diffs = []
    for U in (0.4, 0.2):
        chans, sig = O.pt2_state(g, U, 1.0, T, q, q)
        base = O.FlowOptions(se_iterations=0)
        corr = O.FlowOptions(se_iterations=10, se_atol=0.0, se_rtol=1e-12)
        info = {}
        _, s0 = O.mfrg_rhs(g, U, T, 1.0, 3, q, q, chans, sig, base)
        _, s1 = O.mfrg_rhs(g, U, T, 1.0, 3, q, q, chans, sig, corr, info)
        assert info["se_iterations"] < 10
        diffs.append(np.abs(s1 - s0).max() / np.abs(s0).max())
        _, s2 = O.mfrg_rhs(g, U, T, 1.0, 2, q, q, chans, sig, corr)
        _, s3 = O.mfrg_rhs(g, U, T, 1.0, 2, q, q, chans, sig, base)
        assert np.abs(s2 - s3).max() == 0.0
    # relative to Sigma_dot ~ U^2: the correction ratio falls by 2^2 = 4 (U^4 / U^2)
    assert 3.3 < diffs[0] / diffs[1] < 4.8, diffs


def test_anderson_accelerated_self_energy_corrections_reach_the_same_fixed_point():
    """Anderson acceleration of the self-energy correction iterations (Sec. mfRG) changes the
    path, not the fixed point: at a tight tolerance the accelerated iteration ends at the plain
    one's Sigma_dot and vertex flow, in no more iterations (fewer at depth 4, U = 2)."""
    g, q = O.Grid(9), O.Quad(31)
    ch, sg = O.pt2_state(g, 2.0, 1.0, T, q, q)
    out = {}
    for m in (0, 4):
        info = {}
        fo = O.FlowOptions(se_iterations=40, se_atol=0.0, se_rtol=1e-12, se_anderson=m)
        gd, sd = O.mfrg_rhs(g, 2.0, T, 1.0, 4, q, q, ch, sg, fo, info)
        out[m] = (gd, sd, info["se_iterations"])
    assert np.abs(out[4][1] - out[0][1]).max() < 1e-10 * np.abs(out[0][1]).max()
    for r in range(3):
        a, b = out[4][0][r].K3, out[0][0][r].K3
        assert np.abs(a - b).max() < 1e-9 * np.abs(b).max()
    assert out[4][2] < out[0][2] < 40
