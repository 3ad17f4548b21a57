"""Pins of the oracle's Hartree term (Sec. Hartree-Fock, Eq. Hartree): the occupation of a
Lorentzian level against its closed form at finite temperature (digamma function), the
self-consistent term at particle-hole symmetry, the Friedel sum rule as T -> 0, and the
one-shot term with a dynamic self-energy against an independent adaptive integration, and
the asymmetric parquet solver at eps_d = -U/2 reproducing the particle-hole symmetric one.""" 
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
