"""Pins of the FP64 CPU oracle against what mathematics and the paper fix.

Each test names the passage it follows.  None of them re-types the oracle's own
formula: they compare with closed forms (digamma sums of the bare bubble), an
independent spectral representation of the second-order self-energy, exact
invariants (fluctuation-dissipation relations, causality, crossing and
particle-hole symmetry), finite differences, library routines, and a brute-force
compound-index evaluation of the bubble on tiny grids.
"""
import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

import oracle as O
from workload import random_channel

D, T, U = 1.0, 0.1, 1.0


# ---------------------------------------------------------------- closed forms
def _I(a, b, T):
    """int dv/(2 pi i) tanh(v/2T)/((v-a)(v-b)) closed in the upper half plane: poles of the
    rational part plus the fermionic Matsubara poles of tanh (residue 2T), summed by digamma."""
    r = 0.0
    if a.imag > 0:
        r += np.tanh(a / (2 * T)) / (a - b)
    if b.imag > 0:
        r += np.tanh(b / (2 * T)) / (b - a)
    r += 1.0 / (np.pi * 1j * (a - b)) * (sp.psi(0.5 + 1j * b / (2 * np.pi * T)) - sp.psi(0.5 + 1j * a / (2 * np.pi * T)))
    return r


def bare_B(X, Y, w, Dl=D, T=T):
    """B^{XY}(w) = int dv/(2 pi i) G^X(v + w/2) G^Y(v - w/2), Lorentzian G^R = 1/(v + i Delta),
    G^K = tanh(v/2T)(G^R - G^A)."""
    iD = 1j * Dl
    if (X, Y) == ("R", "A"):
        return 1.0 / (w + 2j * Dl)
    if (X, Y) == ("A", "R"):
        return 1.0 / (2j * Dl - w)
    if X == Y and X in "RA":
        return 0.0
    if (X, Y) == ("R", "K"):
        return _I(-iD, -w - iD, T) - _I(iD, -w - iD, T)
    if (X, Y) == ("A", "K"):
        return _I(-iD, -w + iD, T) - _I(iD, -w + iD, T)
    if (X, Y) == ("K", "R"):
        return _I(-iD, w - iD, T) - _I(iD, w - iD, T)
    if (X, Y) == ("K", "A"):
        return _I(-iD, w + iD, T) - _I(iD, w + iD, T)
    # K K: t(+)t(-) = 1 + coth(w/2T)(t(-) - t(+)) reduces it to the others
    c = 1.0 / np.tanh(w / (2 * T))
    one = -(bare_B("R", "A", w) + bare_B("A", "R", w))
    # int t(-) dG(+) dG(-) = B^{dG,K} and int t(+) dG(+) dG(-) = B^{K,dG}, dG = G^R - G^A
    tm = (bare_B("R", "K", w) - bare_B("A", "K", w))
    tp = (bare_B("K", "R", w) - bare_B("K", "A", w))
    return one + c * (tm - tp)


def _quad_complex(f, lo=-np.inf, hi=np.inf):
    re = si.quad(lambda v: f(v).real, lo, hi, limit=800, epsabs=1e-14, epsrel=1e-12)[0]
    im = si.quad(lambda v: f(v).imag, lo, hi, limit=800, epsabs=1e-14, epsrel=1e-12)[0]
    return re + 1j * im


def _Gc(X, x, Dl=D, T=T):
    GR = 1.0 / (x + 1j * Dl)
    GA = np.conj(GR)
    return {"R": GR, "A": GA, "K": np.tanh(x / (2 * T)) * (GR - GA)}[X]


# ---------------------------------------------------------------- grids & quadrature
def test_gauss_legendre_matches_numpy():
    for n in (1, 2, 7, 64, 201, 2001):
        x = np.zeros(n)
        w = np.zeros(n)
        O.lib().oracle_gauss_legendre(n, x.ctypes.data, w.ctypes.data)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.max(np.abs(x - xr)) < 1e-14
        assert np.max(np.abs(w - wr)) < 1e-14 * max(1.0, n / 100)


def test_grid_map_and_locate():
    g = O.Grid(31, 20.0, 1.0)
    v = g.nodes()
    assert abs(v[0] + 20) < 1e-12 and abs(v[-1] - 20) < 1e-12 and v[15] == 0.0
    assert np.all(np.diff(v) > 0) and np.allclose(v, -v[::-1], atol=1e-13)
    i0, t = O.C.c_int(), O.C.c_double()
    for i in (0, 7, 29, 30):
        assert O.lib().oracle_grid_locate(31, 20.0, 1.0, 0, v[i], O.C.byref(i0), O.C.byref(t)) == 1
        assert i0.value + t.value == pytest.approx(i, abs=1e-9)
    assert O.lib().oracle_grid_locate(31, 20.0, 1.0, 0, 20.5, O.C.byref(i0), O.C.byref(t)) == 0
    # the interpolation variable is the auxiliary x: a point halfway in x gets t = 1/2
    x_mid = (-1 + 2 * 3.5 / 30) * np.arctan(20.0)
    O.lib().oracle_grid_locate(31, 20.0, 1.0, 0, np.tan(x_mid), O.C.byref(i0), O.C.byref(t))
    assert i0.value == 3 and t.value == pytest.approx(0.5, abs=1e-12)


def test_quadrature_maps_integrate_exactly_known_integrals():
    v, w = O.Quad(201, 0, 20.0, 1.0).nodes_weights()
    assert np.sum(w / (1 + v * v)) == pytest.approx(2 * np.arctan(20.0), rel=1e-13)
    assert np.sum(w) == pytest.approx(40.0, rel=1e-12)
    v, w = O.Quad(401, 1, 0.0, 1.0).nodes_weights()
    assert np.sum(w / (1 + v * v)) == pytest.approx(np.pi, rel=1e-13)
    assert np.sum(w / (1 + v * v) ** 2) == pytest.approx(np.pi / 2, rel=1e-12)


# ---------------------------------------------------------------- propagators
def test_propagator_keldysh_structure_and_fdr():
    """G^{1|1} = 0, G^A = (G^R)*, fermionic FDR G^K = 2i tanh(v/2T) Im G^R (Sec. Fluctuation
    dissipation relations), Dyson with a dynamic self-energy."""
    nu = np.linspace(-7, 7, 29)
    g = O.propagator(O.Prop(D, T), nu)
    assert np.all(g[:, 0, 0] == 0)
    assert np.allclose(g[:, 1, 0], 1 / (nu + 1j * D), rtol=1e-15, atol=0)
    assert np.allclose(g[:, 0, 1], np.conj(g[:, 1, 0]), rtol=0, atol=1e-16)
    assert np.allclose(g[:, 1, 1], 2j * np.tanh(nu / (2 * T)) * g[:, 1, 0].imag, rtol=1e-14, atol=1e-16)
    # with a causal dynamic self-energy on a grid: Dyson and the general Keldysh relation
    sg = O.Grid(41, 20.0, 1.0)
    sn = sg.nodes()
    SigR = 0.3 * sn / (sn * sn + 4) - 0.2j / (1 + sn * sn)
    P = O.Prop(D, T, sigma_grid=sg, SigR=SigR)
    gs = O.propagator(P, sn)
    assert np.allclose(gs[:, 1, 0], 1 / (sn + 1j * D - SigR), rtol=1e-14)
    assert np.allclose(gs[:, 1, 1], 2j * np.tanh(sn / (2 * T)) * gs[:, 1, 0].imag, rtol=1e-12, atol=1e-16)


def test_single_scale_is_delta_derivative():
    """S = dG/dDelta at fixed Sigma (Delta-flow, Sec. Flow schemes), S^R = -i (G^R)^2."""
    nu = np.linspace(-5, 5, 23)
    s = O.propagator(O.Prop(D, T), nu, kind=1)
    h = 1e-5
    fd = (O.propagator(O.Prop(D + h, T), nu) - O.propagator(O.Prop(D - h, T), nu)) / (2 * h)
    assert np.allclose(s, fd, rtol=1e-8, atol=1e-10)
    assert np.allclose(s[:, 1, 0], -1j / (nu + 1j * D) ** 2, rtol=1e-14)


# ---------------------------------------------------------------- P1: bare bubble
@pytest.mark.parametrize("w", [0.37, -1.3, 2.5])
def test_bare_bubble_closed_form(w):
    """Pi_a summed with the full-line quadrature equals the digamma closed forms of
    int dv/(2 pi i) G^X(v + w/2) G^Y(v - w/2) placed by the Keldysh structure."""
    # the closed forms themselves agree with adaptive quadrature
    for X, Y in [("R", "K"), ("K", "A"), ("K", "K")]:
        num = _quad_complex(lambda v: _Gc(X, v + w / 2) * _Gc(Y, v - w / 2) / (2j * np.pi))
        assert abs(bare_B(X, Y, w) - num) < 1e-10
    v, wt = O.Quad(2001, 1, 0.0, 1.0).nodes_weights()
    P = O.Prop(D, T)
    pibar = sum(O.bubble_pi(P, 0, w, v[k]) * wt[k] / (2j * np.pi) for k in range(len(v)))
    ktype = {(0, 1): "A", (1, 0): "R", (1, 1): "K"}
    for rp in range(4):
        for cp in range(4):
            a3, a4p = divmod(rp, 2)
            a3p, a4 = divmod(cp, 2)
            X, Y = ktype.get((a3, a3p)), ktype.get((a4, a4p))
            ref = 0.0 if X is None or Y is None else bare_B(X, Y, w)
            assert abs(pibar[rp, cp] - ref) < 2e-8, (rp, cp, pibar[rp, cp], ref)


def test_bare_bubble_p_channel_against_quadrature():
    """Pi_p uses G(w/2 + v) G(w/2 - v): compare with adaptive quadrature of the continuum."""
    w = 0.8
    v, wt = O.Quad(2001, 1, 0.0, 1.0).nodes_weights()
    P = O.Prop(D, T)
    pibar = sum(O.bubble_pi(P, 1, w, v[k]) * wt[k] / (2j * np.pi) for k in range(len(v)))
    ktype = {(0, 1): "A", (1, 0): "R", (1, 1): "K"}
    for rp in range(4):
        for cp in range(4):
            a3, a4 = divmod(rp, 2)
            a3p, a4p = divmod(cp, 2)
            X, Y = ktype.get((a3, a3p)), ktype.get((a4, a4p))
            if X is None or Y is None:
                assert pibar[rp, cp] == 0
                continue
            ref = _quad_complex(lambda x: _Gc(X, w / 2 + x) * _Gc(Y, w / 2 - x) / (2j * np.pi))
            assert abs(pibar[rp, cp] - ref) < 2e-8


# ---------------------------------------------------------------- P2, P3: PT2 K1
def test_pt2_k1_causal_structure_and_bosonic_fdr():
    """K1_a = Gamma_0 Pibar Gamma_0: the all-classical block vanishes, K1^A = (K1^R)*, and
    the bosonic FDR Im K1^R = -(i/2) tanh(w/2T) K1^K holds (Sec. Fluctuation dissipation
    relations), with the full-line quadrature."""
    g = O.Grid(21, 20.0, 1.0)
    k1 = O.pt2_k1(g, U, O.Prop(D, T), O.Quad(1601, 1, 0.0, 1.0))[0]
    w = g.nodes()
    m = k1[0].reshape(len(w), 4, 4)
    u, v = [0, 3], [1, 2]
    KR = m[:, v][:, :, u]
    KA = m[:, u][:, :, v]
    KK = m[:, v][:, :, v]
    scale = np.abs(m).max()
    assert np.abs(m[:, u][:, :, u]).max() < 1e-9 * scale
    assert np.allclose(KR, KR[:, :1, :1], atol=1e-14 * scale)  # four equal entries
    assert np.allclose(KA, np.conj(KR), atol=1e-12 * scale)
    nz = np.abs(w) > 1e-12
    lhs = KR[nz, 0, 0].imag
    rhs = (-0.5j * np.tanh(w[nz] / (2 * T)) * KK[nz, 0, 0])
    assert np.abs(rhs.imag).max() < 1e-9 * scale
    assert np.allclose(lhs, rhs.real, atol=1e-9 * scale)
    # and the retarded entry is (U^2/4)(B^RK + B^KA)
    for iw in (3, 8, 14):
        ref = U * U / 4 * (bare_B("R", "K", w[iw]) + bare_B("K", "A", w[iw]))
        assert abs(KR[iw, 0, 0] - ref) < 1e-8


def test_pt2_k1_scales_as_u_squared():
    g = O.Grid(11)
    q = O.Quad(101)
    P = O.Prop(D, T)
    k1a = O.pt2_k1(g, 1.0, P, q)
    k1b = O.pt2_k1(g, 2.5, P, q)
    for r in range(3):
        assert np.allclose(k1b[r], 6.25 * k1a[r], rtol=1e-14, atol=1e-18)


# ---------------------------------------------------------------- Hartree loop
def test_loop_reproduces_hartree_shift():
    """-L(Gamma_0, G) in the Keldysh-rotated basis gives Sigma^R = U(<n> - 1/2), the Hartree
    term U<n> of Eq. Hartree minus its constant U/2 (which is absorbed in G_H); this fixes the
    sign of Gamma_0, the loop measure dv/(2 pi i) and the spin sum together."""
    eps = 0.7
    P = O.Prop(D, T, eps=eps)
    g = O.Grid(5)
    L = O.loop(O.bare(g, U), P, O.Quad(4001, 1, 0.0, 1.0))
    sig = -L
    nF = lambda x: 0.5 * (1 - np.tanh(x / (2 * T)))
    A = lambda x: (D / np.pi) / ((x - eps) ** 2 + D * D)
    n = si.quad(lambda x: nF(x) * A(x), -np.inf, np.inf, epsabs=1e-14, epsrel=1e-12, limit=400)[0]
    assert np.allclose(sig[:, 1], U * (n - 0.5), atol=1e-8)
    assert np.allclose(sig[:, 2], U * (n - 0.5), atol=1e-8)
    assert np.abs(sig[:, [0, 3]]).max() < 1e-12


# ---------------------------------------------------------------- P5: PT2 self-energy
def _spectral_im_sigma2(nu, Ul=U, Dl=D, T=T):
    """-Im Sigma^R(v)/pi = U^2 int de1 de2 A1 A2 A3 [f(-e1) f(-e2) f(e3) + f(e1) f(e2) f(-e3)],
    e3 = e1 + e2 - v: the textbook second-order self-energy in spectral form."""
    A = lambda e: (Dl / np.pi) / (e * e + Dl * Dl)
    f = lambda e: 0.5 * (1 - np.tanh(e / (2 * T)))
    g = lambda e2, e1: A(e1) * A(e2) * A(e1 + e2 - nu) * (f(-e1) * f(-e2) * f(e1 + e2 - nu)
                                                          + f(e1) * f(e2) * f(-(e1 + e2 - nu)))
    return -np.pi * Ul * Ul * si.dblquad(g, -80, 80, -80, 80, epsabs=1e-13, epsrel=1e-10)[0]


def test_pt2_self_energy_converges_to_spectral_formula():
    """SDE with Gamma = Gamma_0 equals the second-order self-energy (Sec. PT2: the a-bubble of two
    bare vertices closed with G_H).  The discrete result converges as O(h^2) from the bilinear
    interpolation of the bubble on the grid."""
    errs = []
    for N, Nq in [(31, 201), (61, 401)]:
        g = O.Grid(N)
        q = O.Quad(Nq)
        s = O.sde(O.bare(g, U), O.Prop(D, T), q, q)
        nodes = g.nodes()
        i = N // 2 + 2
        ref = _spectral_im_sigma2(nodes[i])
        errs.append(abs(s[i, 1].imag - ref) / abs(ref))
        ref0 = _spectral_im_sigma2(0.0)
        errs.append(abs(s[N // 2, 1].imag - ref0) / abs(ref0))
    assert errs[2] < 0.01 and errs[3] < 0.01
    assert errs[0] / errs[2] > 2.5 and errs[1] / errs[3] > 2.5


def test_sde_symmetries_fdr_causality():
    """Sigma from the SDE: Im Sigma^R <= 0 (Sec. Causality check), Sigma^{2|2} = 0, Sigma^A = (Sigma^R)*,
    FDR Sigma^K = 2i tanh(v/2T) Im Sigma^R (Sec. Fluctuation dissipation relations), particle-hole
    symmetry Sigma^R(-v) = -(Sigma^R(v))*, exact U^2 scaling at second order.
    For a vertex with only its own-channel K1 the discrete map keeps conjugation and particle-hole
    symmetry exactly; the Keldysh zero and the FDR hold up to the truncation of every class beyond
    the largest grid point (the paper's tail rule), measured at 1e-3 on |v| <= 3."""
    g = O.Grid(61)
    q = O.Quad(801, 1, 0.0, 1.0)
    P = O.Prop(D, T)
    V = O.seeded_vertex(g, U, P, q)
    Va = O.Vertex(g, U, [O.Channel(1.0, V.ch[0].K1), O.Channel(0.0), O.Channel(0.0)])
    s = O.sde(Va, P, q, q)
    nu = g.nodes()
    SR, SK = s[:, 1], s[:, 0]
    scale = np.abs(SR).max()
    inner = np.abs(nu) <= 3
    assert np.all(SR.imag <= 1e-12 * scale)
    assert np.allclose(s[:, 2], np.conj(SR), atol=1e-14 * scale)
    assert np.allclose(SR[::-1], -np.conj(SR), atol=1e-13 * scale)
    assert np.abs(s[inner, 3]).max() < 3e-3 * scale
    assert np.abs(SK - 2j * np.tanh(nu / (2 * T)) * SR.imag)[inner].max() < 3e-3 * scale
    s2 = O.sde(O.bare(g, 2.0), P, q, q)
    s1 = O.sde(O.bare(g, 1.0), P, q, q)
    assert np.allclose(s2, 4 * s1, rtol=1e-13, atol=1e-18)


def test_sde_full_seed_residuals_shrink_with_resolution():
    """With all three channels the residuals of conjugation symmetry, the Keldysh zero and the FDR
    come from interpolating the other channels at mapped frequencies and from the cut at +-L; they
    must shrink as the grid is refined, while causality and particle-hole symmetry hold exactly."""
    res = []
    for N, Nq in [(31, 201), (61, 401)]:
        g = O.Grid(N)
        q = O.Quad(Nq)
        P = O.Prop(D, T)
        s = O.sde(O.seeded_vertex(g, U, P, q), P, q, q)
        nu = g.nodes()
        SR = s[:, 1]
        sc = np.abs(SR).max()
        inner = np.abs(nu) <= 3
        assert np.all(SR.imag <= 1e-12 * sc)
        assert np.allclose(SR[::-1], -np.conj(SR), atol=1e-13 * sc)
        res.append([np.abs(s[inner, 2] - np.conj(SR[inner])).max() / sc,
                    np.abs(s[inner, 3]).max() / sc,
                    np.abs(s[inner, 0] - 2j * np.tanh(nu[inner] / (2 * T)) * SR[inner].imag).max() / sc])
    assert max(res[1]) < 0.02
    assert all(b < 0.75 * a for a, b in zip(res[0], res[1]))


def test_sde_rpa_chain_against_continuum():
    """For Gamma = Gamma_0 + K1_a with K1_a = Gamma_0 Pibar Gamma_0, the SDE kernel is
    2 Gamma_0 Pibar Gamma_0 + Gamma_0 Pibar Gamma_0 Pibar Gamma_0 (spin sum 2X + Y); with the
    closed-form Pibar it is integrated densely over |w| <= L and compared with the oracle at
    interior grid nodes (agreement up to the O(h^2) grid interpolation of the bubble)."""
    N = 61
    g = O.Grid(N)
    q = O.Quad(801, 1, 0.0, 1.0)
    P = O.Prop(D, T)
    V = O.seeded_vertex(g, U, P, q)
    Va = O.Vertex(g, U, [O.Channel(1.0, V.ch[0].K1), O.Channel(0.0), O.Channel(0.0)])
    s = O.sde(Va, P, q, q)
    ktype = {(0, 1): "A", (1, 0): "R", (1, 1): "K"}
    u = np.array([1, 0, 0, 1.0])
    vv = np.array([0, 1, 1, 0.0])
    G0 = -(U / 2) * (np.outer(u, vv) + np.outer(vv, u))
    x, wx = np.polynomial.legendre.leggauss(3000)
    om, wt = 20 * x, 20 * wx
    ker = np.zeros((len(om), 4, 4), complex)
    for n_, o in enumerate(om):
        pb = np.zeros((4, 4), complex)
        for rp in range(4):
            for cp in range(4):
                a3, a4p = divmod(rp, 2)
                a3p, a4 = divmod(cp, 2)
                X, Y = ktype.get((a3, a3p)), ktype.get((a4, a4p))
                if X and Y:
                    pb[rp, cp] = bare_B(X, Y, o)
        ker[n_] = 2 * G0 @ pb @ G0 + G0 @ pb @ G0 @ pb @ G0
    nodes = g.nodes()
    for i in (30, 33, 40, 50):
        x2 = nodes[i] - om
        GR = 1 / (x2 + 1j * D)
        GK = np.tanh(x2 / (2 * T)) * (GR - np.conj(GR))
        Gm = np.zeros((len(om), 2, 2), complex)
        Gm[:, 0, 1], Gm[:, 1, 0], Gm[:, 1, 1] = np.conj(GR), GR, GK
        ref = np.zeros((2, 2), complex)
        for a1p in range(2):
            for a1 in range(2):
                for a2 in range(2):
                    for a2p in range(2):
                        f = 4 * (2 * a1p + a2) + (2 * a1 + a2p)
                        ref[a1p, a1] += np.sum(-0.5 * wt / (2j * np.pi) * ker[:, f // 4, f % 4] * Gm[:, a2, a2p])
        assert abs(s[i, 1] - ref[0, 1]) < 0.01 * abs(ref[0, 1])


# ---------------------------------------------------------------- P6: susceptibility
def test_chi_bare_vertex_closed_form_and_sign():
    """With Gamma = Gamma_0: chi^R = P^R - (U/2)(P^R)^2 for the X (transverse spin) combination
    and P^R + (U/2)(P^R)^2 for D = X + 2Y (density): spin enhanced, density suppressed for
    repulsive U, which fixes the sign of Gamma_0 relative to the bubble."""
    g = O.Grid(9)
    q = O.Quad(1201, 1, 0.0, 1.0)
    ch = O.chi(O.bare(g, U), O.Prop(D, T), q)
    w = g.nodes()
    cx = O.chi_scalar(ch[0])
    cd = O.chi_scalar(ch[1])
    for iw in range(len(w)):
        PR = bare_B("R", "K", w[iw]) + bare_B("K", "A", w[iw]) if abs(w[iw]) > 1e-12 else None
        if PR is None:
            continue
        assert abs(cx[iw] - (PR - U / 2 * PR * PR)) < 5e-7  # full-line quadrature error at |w| = L
        assert abs(cd[iw] - (PR + U / 2 * PR * PR)) < 5e-7
    i0 = len(w) // 2
    P0 = O.chi_scalar(O.chi(O.bare(g, 0.0), O.Prop(D, T), q)[0])[i0]
    assert P0.real < 0 and abs(cx[i0]) > abs(P0) > abs(cd[i0])


def test_chi_of_every_channel_factorises_for_the_bare_vertex_and_diagonalises_its_bubble():
    """With Gamma = Gamma_0 (constant in the fermionic frequencies) the double sum of the
    susceptibility factorises exactly: chi_r^c = S_r + S_r Gamma_0^c S_r with S_r = chi_r at
    U = 0, the sum of the weighted pair bubbles.  The same S_r builds the one-loop K1 class of the
    Bethe-Salpeter bubble (itself pinned by closed forms and crossing symmetry):
    B_r(Gamma_0, Gamma_0)^c = pref_r Gamma_0^c S_r Gamma_0^c with the channel prefactors +1, 1/2,
    -1 -- which holds only when the two spin combinations c are the ones that diagonalise channel
    r's spin sum (a: X, X + 2Y; p: X + Y, X - Y; t: Y, 2X + Y), and only when chi uses channel r's
    bubble and pair order."""
    g = O.Grid(7)
    q = O.Quad(61)
    P = O.Prop(D, T)
    g0, zero = O.bare(g, U), O.bare(g, 0.0)
    w = g.nodes()
    combos = {0: ((1, 0), (1, 2)), 1: ((1, 1), (1, -1)), 2: ((0, 1), (2, 1))}
    pref = (1.0, 0.5, -1.0)
    for r in range(3):
        S = O.chi_channel(r, zero, P, q)
        assert np.abs(S[0] - S[1]).max() == 0.0
        ch = O.chi_channel(r, g0, P, q)
        K1 = O.bubble(r, g0, g0, P, q).K1
        XY = O.vertex_eval(g0, r, [(wi, 0.37, -1.3) for wi in w])
        for c, (mx, my) in enumerate(combos[r]):
            for i in range(len(w)):
                Gc = (mx * XY[i, 0] + my * XY[i, 1]).reshape(4, 4)
                Sm = S[0, i].reshape(4, 4)
                scale = np.abs(Sm).max()
                assert scale > 1e-3
                assert np.abs(ch[c, i].reshape(4, 4) - (Sm + Sm @ Gc @ Sm)).max() < 1e-13
                k1 = (mx * K1[0][i] + my * K1[1][i]).reshape(4, 4)
                assert np.abs(k1 - pref[r] * Gc @ Sm @ Gc).max() < 1e-13
    # channel a is the susceptibility of the Schwinger-Dyson path
    assert np.abs(O.chi_channel(0, g0, P, q) - O.chi(g0, P, q)).max() == 0.0


# ---------------------------------------------------------------- P7: crossing symmetry
def _legs_grid(n):
    rng = np.random.default_rng(5)
    pts = []
    for _ in range(n):
        n1p, n2p, n1 = rng.uniform(-6, 6, 3)
        n2 = n1p + n2p - n1
        pts.append((n1p, n2p, n1, n2))
    return np.array(pts)


def test_crossing_symmetry_of_bubble_sum():
    """Gamma(1'2'|21) = -Gamma(1'2'|12) (antisymmetry of the vertex under exchange of two
    incoming legs, Sec. Symmetries) for Gamma' = Gamma_0 + sum_r B_r(Gamma, Gamma), where
    Gamma = Gamma_0 + sum_r B_r(Gamma_0, Gamma_0) is itself crossing symmetric.  Crossing maps
    the a channel onto t and p onto itself, so this checks the channel parametrisations,
    prefactors, Keldysh pair orders and spin sums of all three bubbles together."""
    g = O.Grid(11, 10.0, 1.0)
    q = O.Quad(61, 0, 10.0, 1.0)
    P = O.Prop(D, T)
    g0 = O.bare(g, U)
    V1 = O.combine(g, [(r, O.bubble(r, g0, g0, P, q), 1.0) for r in range(3)], r0=U)
    V2 = O.combine(g, [(r, O.bubble(r, V1, V1, P, q), 1.0) for r in range(3)], r0=U)
    legs = _legs_grid(12)
    al, sg, nu, alx, sgx, nux = [], [], [], [], [], []
    for L in legs:
        for kel in range(16):
            a = [(kel >> b) & 1 for b in range(4)]
            for s in ([0, 1, 0, 1], [0, 1, 1, 0], [0, 0, 0, 0]):
                al.append(a); sg.append(s); nu.append(L)
                alx.append([a[0], a[1], a[3], a[2]]); sgx.append([s[0], s[1], s[3], s[2]])
                nux.append([L[0], L[1], L[3], L[2]])
    for V in (V1, V2):
        x = O.vertex_legs(V, al, sg, nu)
        y = O.vertex_legs(V, alx, sgx, nux)
        scale = np.abs(x).max()
        assert scale > 1e-3
        assert np.abs(x + y).max() < 1e-12 * scale


def test_particle_hole_symmetry_of_k1():
    """At particle-hole symmetry the bare bubble satisfies Pibar(-w) = Pibar(w)^* entry-wise up to
    the Keldysh structure; for K1 this gives K1^R(-w) = K1^R(w)^* (real part even, imaginary odd)."""
    g = O.Grid(15)
    k1 = O.pt2_k1(g, U, O.Prop(D, T), O.Quad(301))[0][0].reshape(15, 4, 4)
    KR = k1[:, 1, 0]
    assert np.allclose(KR[::-1], np.conj(KR), atol=1e-14 * np.abs(KR).max())


# ---------------------------------------------------------------- P9, P10: brute force
@pytest.mark.parametrize("r", [0, 1, 2])
@pytest.mark.parametrize("kind", [0, 1])
def test_pair_matrix_bubble_equals_compound_index_sum(r, kind):
    """The K-class pair-matrix form of B_r (literal spin sums, Gamma split into its v->infinity
    limit and remainder) sums to the defining 8-fold compound-index sum over internal Keldysh
    and spin indices, evaluated with a leg-based vertex (tiny grids, all classes random)."""
    n = 5
    g = O.Grid(n, 6.0, 1.0)
    q = O.Quad(7, 0, 6.0, 1.0)
    P = O.Prop(D, 0.3)
    chans = []
    for rr in range(3):
        rc = random_channel(n, 100 + rr, 0.3)
        chans.append(O.Channel(1.0 - 0.25 * rr, rc["K1"], rc["K2"], rc["K2p"], rc["K3"]))
    Lv = O.Vertex(g, 0.7, chans)
    chans2 = []
    for rr in range(3):
        rc = random_channel(n, 200 + rr, 0.3)
        chans2.append(O.Channel(1.0, rc["K1"], rc["K2"], rc["K2p"], rc["K3"]))
    Rv = O.Vertex(g, 0.7, chans2)
    out = O.bubble(r, Lv, Rv, P, q, kind)
    nodes = g.nodes()
    for (iw, i, j) in [(2, 1, 3), (0, 4, 2), (3, 2, 2), (4, 0, 0)]:
        tot = out.K1[:, iw] + out.K2[:, iw, i] + out.K2p[:, iw, j] + out.K3[:, iw, i, j]
        ref = O.bubble_brute(r, Lv, Rv, P, q, nodes[iw], nodes[i], nodes[j], kind)
        assert np.abs(tot - ref).max() < 1e-13 * np.abs(ref).max()


def test_bubble_points_match_full_arrays():
    n = 7
    g = O.Grid(n, 8.0, 1.0)
    q = O.Quad(15, 0, 8.0, 1.0)
    P = O.Prop(D, T)
    rc = [random_channel(n, 300 + rr, 0.1) for rr in range(3)]
    V = O.Vertex(g, U, [O.Channel(1.0, c["K1"], c["K2"], c["K2p"], c["K3"]) for c in rc])
    for r in range(3):
        full = O.bubble(r, V, V, P, q)
        pts = [(8, 2, 3, 4), (2, 5, 1, 0), (4, 0, 0, 6), (1, 6, 0, 0)]
        got = O.bubble_points(r, V, V, P, q, pts)
        ref = [full.K3[:, 2, 3, 4], full.K2[:, 5, 1], full.K2p[:, 0, 6], full.K1[:, 6]]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


# ---------------------------------------------------------------- P11: multiloop
def test_one_loop_insertion_is_delta_derivative_of_pt2():
    """With Gamma = Gamma_0 the one-loop flow term B_r(Gamma_0, Gamma_0; Pidot) with
    Pidot = S G + G S (Eq. 1l) is the Delta-derivative of the PT2 vertex."""
    g = O.Grid(9)
    q = O.Quad(81)
    P = O.Prop(D, T)
    g0 = O.bare(g, U)
    h = 1e-5
    for r in range(3):
        d1 = O.bubble(r, g0, g0, P, q, kind=1, cmask=O.C_K1).K1
        kp = O.bubble(r, g0, g0, O.Prop(D + h, T), q, cmask=O.C_K1).K1
        km = O.bubble(r, g0, g0, O.Prop(D - h, T), q, cmask=O.C_K1).K1
        fd = (kp - km) / (2 * h)
        assert np.abs(d1 - fd).max() < 1e-8 * np.abs(d1).max()


def test_multiloop_orders_scale_as_powers_of_U():
    """Every multiloop order l is (l+1)-linear in the vertex, so for Gamma = Gamma_0 it scales
    as U^(l+1) (Eqs. 1l-3l); at l = 1 the insertion of the bare vertex has K1 only."""
    g = O.Grid(7, 8.0, 1.0)
    q = O.Quad(21, 0, 8.0, 1.0)
    P = O.Prop(D, T)
    o1 = O.mloop(O.bare(g, 1.0), P, q, 3)
    o2 = O.mloop(O.bare(g, 2.0), P, q, 3)
    for ell in range(3):
        for r in range(3):
            for c in ("K1", "K2", "K2p", "K3"):
                a, b = getattr(o1[ell][r], c), getattr(o2[ell][r], c)
                assert np.allclose(b, 2.0 ** (ell + 2) * a, rtol=1e-12, atol=1e-300)
    assert all(np.abs(getattr(o1[0][r], c)).max() == 0.0 for r in range(3) for c in ("K2", "K2p", "K3"))


# The multiloop pins below take the insertions from a multiloop implementation passed in
# (O.mloop itself, or a copy with a planted mistake in the mutation test), so that what they
# pin is that code, not a hand composition of bubbles.
def _chan_add(*chs):
    return O.Channel(1.0, *[sum(getattr(c, k) for c in chs) for k in ("K1", "K2", "K2p", "K3")])


def _eps_dual(arr):
    """Dual array with value 0 and derivative arr: a vertex Gamma_0 + eps*gamma evaluated with it
    gives, in the derivative part, exactly the term of a multilinear map linear in gamma."""
    d = np.zeros(arr.shape + (4,))
    d[..., 1] = arr.real
    d[..., 3] = arr.imag
    return d


def _parquet_orders(g, q, Ul):
    """Orders U^2, U^3, U^4 of the parquet vertex in the parquet approximation (R = Gamma_0,
    Bethe-Salpeter equations gamma_r = B_r(I_r, Gamma), I_r = Gamma_0 + sum_{r' != r} gamma_r',
    Gamma = Gamma_0 + sum_r gamma_r; Sec. parquet solver) with Sigma = 0, as dual arrays carrying
    their Delta-derivative: gamma^(2)_r = B_r(G0, G0), gamma^(3)_r = B_r(G0, Gamma^(2)) +
    B_r(I^(2)_r, G0), gamma^(4)_r = B_r(G0, Gamma^(3)) + B_r(I^(2)_r, Gamma^(2)) + B_r(I^(3)_r, G0)."""
    Pd = O.Prop(D, T, dDelta=1.0)
    g0 = O.bare(g, Ul)

    def vert(chs, skip=None):
        return O.Vertex(g, 0.0, [O.Channel(0.0) if rr == skip else chs[rr] for rr in range(3)])

    def B(r, a, b):
        return O.bubble(r, a, b, Pd, q, 0, O.C_ALL, dual=True)

    g2 = [B(r, g0, g0) for r in range(3)]
    g3 = [_chan_add(B(r, g0, vert(g2)), B(r, vert(g2, r), g0)) for r in range(3)]
    g4 = [_chan_add(B(r, g0, vert(g3)), B(r, vert(g2, r), vert(g2)), B(r, vert(g3, r), g0)) for r in range(3)]
    return g2, g3, g4


def _value(ch):
    return O.Channel(1.0, *[O.dual_parts(getattr(ch, k))[0] for k in ("K1", "K2", "K2p", "K3")])


def _deriv(ch):
    return O.Channel(1.0, *[O.dual_parts(getattr(ch, k))[1] for k in ("K1", "K2", "K2p", "K3")])


def _rel_max(a_list, b_list):
    """max over channels and classes of |a - b|_inf / max |b|_inf."""
    scale = max(np.abs(getattr(b, k)).max() for b in b_list for k in ("K1", "K2", "K2p", "K3"))
    assert scale > 0
    return max(np.abs(getattr(a, k) - getattr(b, k)).max() for a, b in zip(a_list, b_list)
               for k in ("K1", "K2", "K2p", "K3")) / scale


def _total_derivative_residuals(mloop, g, q, Ul=U):
    """The multiloop flow equations (Sec. mfRG, Eqs. 1l-3l) summed over l reproduce the total
    Delta-derivative of the parquet vertex (with Sigma fixed, no Katanin term).  Order by order in
    U, with Gamma = Gamma_0 + gamma^(2) + gamma^(3) and f_l the l-loop insertion (an (l+1)-linear
    map of Gamma):
      U^3:  d gamma^(3)/dDelta = [f_1 linear in gamma^(2) at Gamma_0] + f_2(Gamma_0),
      U^4:  d gamma^(4)/dDelta = [f_1 linear in gamma^(3)] + f_1(gamma^(2)) + [f_2 linear in
            gamma^(2)] + f_3(Gamma_0),
    where "linear in gamma" is the derivative part of f_l(Gamma_0 + eps gamma) with dual numbers.
    Returns the relative residuals (third order, fourth order)."""
    P = O.Prop(D, T)
    g2d, g3d, g4d = _parquet_orders(g, q, Ul)
    g2 = [_value(c) for c in g2d]
    g3 = [_value(c) for c in g3d]

    def eps_vertex(chs):
        return O.Vertex(g, Ul, [O.Channel(1.0, *[_eps_dual(getattr(c, k)) for k in ("K1", "K2", "K2p", "K3")])
                                for c in chs])

    f_bare = mloop(O.bare(g, Ul), P, q, 3)
    f_g2 = mloop(eps_vertex(g2), P, q, 2, dual=True)
    f_g3 = mloop(eps_vertex(g3), P, q, 1, dual=True)
    f1_g2g2 = mloop(O.Vertex(g, 0.0, g2), P, q, 1)
    m3 = [_chan_add(_deriv(f_g2[0][r]), f_bare[1][r]) for r in range(3)]
    m4 = [_chan_add(_deriv(f_g3[0][r]), f1_g2g2[0][r], _deriv(f_g2[1][r]), f_bare[2][r]) for r in range(3)]
    return (_rel_max(m3, [_deriv(c) for c in g3d]), _rel_max(m4, [_deriv(c) for c in g4d]))


def _grid_rule(n, L=20.0, a=1.0):
    return O.Quad(n, 2, L, a)


def test_grid_node_rule_is_a_quadrature_on_the_grid():
    """The rule used by the fourth-order pin: its nodes are the grid's nodes, and it integrates
    1/(1 + v^2) over [-L, L] (a linear function of the auxiliary variable, exact for the
    trapezoid rule) to 2 atan(L)."""
    g = O.Grid(9)
    v, w = _grid_rule(9).nodes_weights()
    assert np.array_equal(v, g.nodes())
    assert abs(np.sum(w / (1 + v * v)) - 2 * np.arctan(20.0)) < 1e-14


def test_multiloop_total_derivative_at_third_and_fourth_order():
    """The multiloop insertions of O.mloop reproduce the total Delta-derivative of the parquet
    vertex at third order (l = 1, 2) and fourth order (l = 1, 2, 3 with the centre term) in U.
    Both identities are exact in the discrete scheme when the within-channel compositions
    associate: at third order every own-channel object is a K1 (a matrix per transfer frequency),
    so any Gauss-Legendre rule will do; at fourth order own-channel K2/K2' objects are read back
    at the loop frequencies, which associates exactly only when the loop frequencies are grid
    nodes (then every bubble is a plain matrix product over the nodes), hence the grid-node rule.
    With Gauss-Legendre nodes the fourth-order residual is the interpolation error of those
    reads (O(h^2)), not zero."""
    g = O.Grid(9)
    r3, _ = _total_derivative_residuals(O.mloop, g, O.Quad(31))
    assert r3 < 1e-12
    r3, r4 = _total_derivative_residuals(O.mloop, g, _grid_rule(9))
    assert r3 < 1e-12 and r4 < 1e-12, (r3, r4)


def _mirror_residual(mloop, eps=0.0):
    """At l = 2 the insertion of Gamma_0 is L + R with L = B_r(gdot_rbar, Gamma_0) (class K2 only)
    and R = B_r(Gamma_0, gdot_rbar) (K2' only).  Reading the bubble with its two sides exchanged
    maps L onto R: in the t channel K2'(w, v) = K2(-w, v)^T in the Keldysh pair indices; in a and p
    this holds combined with particle-hole symmetry, K2'(w, v) = K2(-w, -v)^T."""
    g = O.Grid(7, 8.0, 1.0)
    q = O.Quad(21, 0, 8.0, 1.0)
    o = mloop(O.bare(g, 1.0), O.Prop(D, T, eps=eps), q, 2)[1]
    res = 0.0
    for r in (range(3) if eps == 0.0 else (2,)):
        A = o[r].K2.reshape(2, 7, 7, 4, 4).transpose(0, 1, 2, 4, 3)[:, ::-1]
        if r != 2:
            A = A[:, :, ::-1]
        Bm = o[r].K2p.reshape(2, 7, 7, 4, 4)
        scale = max(np.abs(Bm).max(), np.abs(A).max())
        assert scale > 0
        # K1 and K3 must vanish: neither insertion has a part constant in both fermionic arguments
        res = max(res, np.abs(A - Bm).max() / scale, np.abs(o[r].K1).max() / scale,
                  np.abs(o[r].K3).max() / scale)
    return res


def test_multiloop_l2_left_and_right_insertions_are_mirror_images():
    assert _mirror_residual(O.mloop) < 1e-13
    assert _mirror_residual(O.mloop, eps=0.3) < 1e-13


def _mloop_with_mistake(mistake):
    """A copy of the oracle's multiloop recursion with one planted mistake (CPU only)."""
    def mloop(V, P, q, nloops, dual=False, centres=None):
        g = V.grid
        out = []
        for ell in range(1, nloops + 1):
            this = []
            for r in range(3):
                if ell == 1:
                    this.append(O.bubble(r, V, V, P, q, 1, O.C_ALL, dual))
                    continue
                prev = out[ell - 2]
                others = [rr for rr in range(3) if rr != r or mistake == "rbar_includes_r"]
                rbar = O.combine(g, [(rr, prev[rr], 1.0) for rr in others])
                if mistake == "right_insertion_twice":
                    Lt = O.bubble(r, V, rbar, P, q, 0, O.C_ALL, dual)
                else:
                    Lt = O.bubble(r, rbar, V, P, q, 0, O.C_ALL, dual)
                Rt = O.bubble(r, V, rbar, P, q, 0, O.C_ALL, dual)
                tot = _chan_add(Lt, Rt)
                if ell >= 3:
                    prev2 = out[ell - 2] if mistake == "centre_from_previous_order" else out[ell - 3]
                    rbar2 = O.combine(g, [(rr, prev2[rr], 1.0) for rr in range(3) if rr != r])
                    if mistake == "centre_inner_mirrored":
                        inner = O.bubble(r, V, rbar2, P, q, 0, O.C_ALL, dual)
                    else:
                        inner = O.bubble(r, rbar2, V, P, q, 0, O.C_ALL, dual)
                    iv = O.combine(g, [(r, inner, 1.0)])
                    if mistake == "centre_outer_mirrored":
                        Ct = O.bubble(r, iv, V, P, q, 0, O.C_ALL, dual)
                    else:
                        Ct = O.bubble(r, V, iv, P, q, 0, O.C_ALL, dual)
                    tot = _chan_add(tot, Ct)
                this.append(tot)
            out.append(this)
        return out
    return mloop


@pytest.mark.parametrize("mistake", ["none", "rbar_includes_r", "right_insertion_twice",
                                     "centre_from_previous_order", "centre_inner_mirrored",
                                     "centre_outer_mirrored"])
def test_multiloop_pins_catch_planted_mistakes(mistake):
    """The multiloop pins above detect each plausible mistake in the recursion: the channel sum
    rbar containing r itself, the left insertion replaced by a second right one, the centre term
    built from order l-1 instead of l-2, or its inner or outer bubble with the sides exchanged."""
    f = _mloop_with_mistake(mistake)
    r3, r4 = _total_derivative_residuals(f, O.Grid(9), _grid_rule(9))
    mirror = _mirror_residual(f)
    worst = max(r3, r4, mirror)
    if mistake == "none":
        assert worst < 1e-12
    else:
        assert worst > 1e-3, (r3, r4, mirror)


# ---------------------------------------------------------------- P13: sum rule
def test_spectral_sum_rule_with_dyson_self_energy():
    """int A(v) dv = 1 (Sec. Sum rule for the spectral function) for G^R = 1/(v + i Delta - Sigma^R)
    with a causal self-energy given on a grid: exact for an analytic Sigma up to its linear
    interpolation (shrinking with the grid), and approached by the interpolated SDE self-energy."""
    v, w = O.Quad(8001, 1, 0.0, 1.0).nodes_weights()
    dev = []
    for N in (101, 401):
        g = O.Grid(N, 200.0, 1.0)
        sn = g.nodes()
        P = O.Prop(D, T, sigma_grid=g, SigR=0.5 / (sn + 2j))
        GR = O.propagator(P, v)[:, 1, 0]
        dev.append(abs(np.sum(w * (-GR.imag / np.pi)) - 1.0))
    assert dev[1] < 1e-7 and dev[1] < 0.25 * dev[0]
    dev = []
    for N in (31, 61):
        g = O.Grid(N)
        q = O.Quad(10 * N - 9)
        s = O.sde(O.bare(g, 2.0), O.Prop(D, T), q, q)
        P = O.Prop(D, T, sigma_grid=g, SigR=s[:, 1].copy())
        GR = O.propagator(P, v)[:, 1, 0]
        dev.append(abs(np.sum(w * (-GR.imag / np.pi)) - 1.0))
    assert dev[1] < 2e-3 and dev[1] < dev[0]


# ---------------------------------------------------------------- P14: exact derivatives
def test_dual_numbers_match_finite_differences():
    """The forward-mode dual evaluation of the discrete SDE map (seed -> Sigma) agrees with
    central finite differences in U and Delta."""
    g = O.Grid(9)
    q = O.Quad(41)

    def sigma(Ul, Dl, dual=False, dU=0.0, dD=0.0):
        P = O.Prop(Dl, T, dDelta=dD)
        V = O.seeded_vertex(g, Ul, P, q, dual=dual, dU=dU)
        return O.sde(V, P, q, q, dual=dual)

    d = sigma(U, D, True, dU=1.0)
    dU_exact = d[..., 1] + 1j * d[..., 3]
    h = 1e-5
    fdU = (sigma(U + h, D) - sigma(U - h, D)) / (2 * h)
    assert np.allclose(d[..., 0] + 1j * d[..., 2], sigma(U, D), rtol=1e-14, atol=1e-18)
    assert np.abs(dU_exact - fdU).max() < 1e-7 * np.abs(dU_exact).max()
    d = sigma(U, D, True, dD=1.0)
    dD_exact = d[..., 1] + 1j * d[..., 3]
    fdD = (sigma(U, D + h) - sigma(U, D - h)) / (2 * h)
    assert np.abs(dD_exact - fdD).max() < 1e-7 * np.abs(dD_exact).max()


# ---------------------------------------------------------------- parquet solver
def _crossing_residual(V):
    legs = _legs_grid(10)
    al, sg, nu, alx, sgx, nux = [], [], [], [], [], []
    for L in legs:
        for kel in range(16):
            a = [(kel >> b) & 1 for b in range(4)]
            for s in ([0, 1, 0, 1], [0, 1, 1, 0]):
                al.append(a); sg.append(s); nu.append(L)
                alx.append([a[0], a[1], a[3], a[2]]); sgx.append([s[0], s[1], s[3], s[2]])
                nux.append([L[0], L[1], L[3], L[2]])
    x = O.vertex_legs(V, al, sg, nu)
    y = O.vertex_legs(V, alx, sgx, nux)
    return np.abs(x + y).max() / np.abs(x).max()


def test_parquet_third_order_expansion():
    """The converged parquet state, expanded in U, starts with the second- and third-order
    diagrams (Sec. parquet solver; PT2 Sec.): gamma_r = gamma_r^(2) + gamma_r^(3) + O(U^4) with
    gamma_r^(3) = 1/2 [B_r(Gamma_0, Gamma^(2)) + B_r(I_r^(2), Gamma_0) + B_r(Gamma_0, I_r^(2))
    + B_r(Gamma^(2), Gamma_0)] (the symmetrized BSE at third order), and
    Sigma = Sigma^(2) + Sigma^(3) + O(U^4) with Sigma^(3) = -1/2 L(B_a(Gamma_0, Gamma^(2)), G).
    The remainders relative to the third-order terms shrink linearly with U."""
    g, q = O.Grid(9), O.Quad(31)
    P0 = O.Prop(D, T)
    errs = []
    for u in (0.1, 0.05):
        chans, sig, res = O.parquet_solve(g, u, D, T, q, q, alpha=1.0, iterations=40, tol=1e-14)
        assert res[-1] < 1e-13
        g0 = O.bare(g, u)
        k1 = O.pt2_k1(g, u, P0, q)
        all2 = O.Vertex(g, 0.0, [O.Channel(1.0, k1[r]) for r in range(3)])
        e_g = 0.0
        for r in range(3):
            i2 = O.Vertex(g, 0.0, [O.Channel(1.0, k1[rr]) if rr != r else O.Channel(0.0) for rr in range(3)])
            terms = [O.bubble(r, g0, all2, P0, q), O.bubble(r, i2, g0, P0, q), O.bubble(r, g0, i2, P0, q),
                     O.bubble(r, all2, g0, P0, q)]
            for c in ("K1", "K2", "K2p"):
                third = 0.5 * sum(getattr(t_, c) for t_ in terms)
                second = k1[r] if c == "K1" else 0.0
                e_g = max(e_g, np.abs(getattr(chans[r], c) - second - third).max() / np.abs(third).max())
        s2 = O.sde(g0, P0, q, q)
        phi3 = O.bubble(0, g0, all2, P0, q, 0, O.C_K1 | O.C_K2P)
        s3 = -0.5 * O.loop(O.Vertex(g, 0.0, [O.Channel(1.0, phi3.K1, None, phi3.K2p, None), O.Channel(0.0),
                                             O.Channel(0.0)]), P0, q)
        e_s = np.abs(sig - s2 - s3).max() / np.abs(s3).max()
        errs.append((e_g, e_s))
    (g1, s1), (g2, s2_) = errs
    assert g1 < 0.2 and s1 < 0.2
    assert 0.3 < g2 / g1 < 0.7 and 0.3 < s2_ / s1 < 0.7


def test_parquet_iteration_preserves_crossing_and_contracts():
    """From the crossing-symmetric PT2 state every parquet iterate stays crossing symmetric
    (symmetric grids map grid points onto grid points), and with mixing 0.5 at U = 1 the
    relative change per iteration decreases geometrically."""
    g = O.Grid(11, 10.0, 1.0)
    q = O.Quad(61, 0, 10.0, 1.0)
    chans, sig, res = O.parquet_solve(g, U, D, T, q, q, alpha=0.5, iterations=6)
    assert all(b < a for a, b in zip(res[1:], res[2:]))
    assert res[-1] / res[2] < 0.5
    assert _crossing_residual(O.Vertex(g, U, chans)) < 1e-12


# ---------------------------------------------------------------- mfRG flow
def test_flow_of_pt2_vertex_reaches_pt2_at_the_end_to_second_order():
    """The one-loop vertex flow is the Delta-derivative of the PT2 vertex at order U^2 (Eq. 1l),
    so flowing the PT2 state from Delta_i = 2 to Delta_f = 1 reproduces the PT2 vertex at
    Delta_f up to O(U^3) and the Runge-Kutta error: the deviation relative to the PT2 vertex
    falls linearly with U and with the fourth power of the step."""
    g, q = O.Grid(9), O.Quad(31)
    devs = {}
    for u, steps in ((0.1, 4), (0.05, 4), (0.05, 2)):
        chans, sig = O.pt2_state(g, u, 2.0, T, q, q)
        chans, sig, _ = O.mfrg_flow(g, u, T, 2.0, 1.0, steps, 1, q, q, chans, sig)
        ref = O.pt2_k1(g, u, O.Prop(1.0, T), q)
        devs[(u, steps)] = max(np.abs(chans[r].K1 - ref[r]).max() / np.abs(ref[r]).max() for r in range(3))
    d1, d2 = devs[(0.1, 4)], devs[(0.05, 4)]
    assert d1 < 0.05
    assert 0.3 < d2 / d1 < 0.7  # O(U): the remaining deviation is the third order


def test_flow_self_energy_matches_sde_pt2_up_to_discretisation():
    """The one-loop self-energy flow -L(Gamma, S) integrates, at order U^2, to the second-order
    self-energy; the SDE form Sigma^(2) = -1/2 L(B_a(Gamma_0, Gamma_0), G) reads the same
    diagram at other frequencies, so the two agree up to the discretisation, which shrinks
    with the grid."""
    devs = []
    for n, nq in ((9, 31), (17, 81)):
        g, q = O.Grid(n), O.Quad(nq)
        chans, sig = O.pt2_state(g, 0.05, 2.0, T, q, q)
        chans, sig, _ = O.mfrg_flow(g, 0.05, T, 2.0, 1.0, 2, 1, q, q, chans, sig)
        s2 = O.sde(O.bare(g, 0.05), O.Prop(1.0, T), q, q)
        devs.append(np.abs(sig - s2).max() / np.abs(s2).max())
    assert devs[0] < 0.1 and devs[1] < 0.75 * devs[0]


def test_pt2_self_energy_obeys_kramers_kronig():
    """Re Sigma^R(v) = (1/pi) P int dv' Im Sigma^R(v') / (v' - v) (Sec. Kramers-Kronig check), with
    Im Sigma^R interpolated as the method interpolates it and zero beyond the grid; the residual
    is the discretisation and shrinks with the grid."""
    res = []
    for N, Nq in ((41, 301), (81, 601)):
        g = O.Grid(N)
        s = O.sde(O.bare(g, U), O.Prop(D, T), O.Quad(Nq, 1, 0.0, 1.0), O.Quad(Nq, 1, 0.0, 1.0))
        v = g.nodes()
        th = np.arctan(g.L / g.a)
        xs = np.arctan(v / g.a) / th
        im = lambda x: np.interp(np.arctan(x / g.a) / th, xs, s[:, 1].imag)
        worst = 0.0
        for i in range(N // 2 - 6, N // 2 + 7, 3):
            pv = si.quad(im, -g.L, g.L, weight="cauchy", wvar=v[i], limit=2000, epsabs=1e-13)[0] / np.pi
            worst = max(worst, abs(pv - s[i, 1].real))
        res.append(worst / np.abs(s[:, 1]).max())
    assert res[0] < 2e-3 and res[1] < 0.6 * res[0], res
