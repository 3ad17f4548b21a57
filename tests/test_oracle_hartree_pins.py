"""Pins of the oracle's Hartree term (Sec. Hartree-Fock, Eq. Hartree): the occupation of a
Lorentzian level against its closed form at finite temperature (digamma function), the
self-consistent term at particle-hole symmetry, the Friedel sum rule as T -> 0, and the
one-shot term with a dynamic self-energy against an independent adaptive integration."""
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
    nF = lambda x: 0.5 * (1 - np.tanh(x / (2 * T)))
    f = lambda x: -nF(x) * (1.0 / (x - E + 1j * D - sig_at(x))).imag / np.pi
    pts = [-g.L, -2, -1, 0, 1, 2, g.L]
    n = sum(si.quad(f, a, b, epsabs=1e-13, epsrel=1e-12, limit=400)[0] for a, b in zip(pts[:-1], pts[1:]))
    n += si.quad(f, -np.inf, -g.L, epsabs=1e-14, limit=200)[0] + si.quad(f, g.L, np.inf, epsabs=1e-14, limit=200)[0]
    got, _ = O.hartree(U, eps_d, D, T, O.Quad(20001, 1, 0.0, 1.0), g, sig, self_consistent=False, sigma_H=sH)
    assert abs(got - U * n) < 1e-6 * U
