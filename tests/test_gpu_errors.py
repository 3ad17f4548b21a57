"""Host-side argument checks of the flow, parquet, Hartree, adaptive and loop entry points: every
case is rejected before any launch with KqftError (no kernel runs on invalid input)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

D, T = 1.0, 0.1


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def _state(K, n):
    chans = [K.alloc_channel(n) for _ in range(3)]
    return chans, torch.zeros((n, 4), dtype=torch.complex128, device="cuda")


def test_flow_arguments():
    K = _K()
    n = 5
    g, q = K.Grid(n), K.Quad(11)
    for fo, li, lf in ((K.FlowOptions(reg=7), 2.0, 1.0),                     # unknown regulator
                       (K.FlowOptions(reg=K.REG_U, Delta=1.0), 0.0, 1.0),     # lambda must be positive
                       (K.FlowOptions(reg=K.REG_NU, Delta=-1.0), 1.0, 0.5),   # Delta of the bath
                       (K.FlowOptions(adaptive=True, atol=0.0, rtol=0.0), 2.0, 1.0),
                       (K.FlowOptions(adaptive=True, max_steps=0), 2.0, 1.0),
                       (K.FlowOptions(se_iterations=-1), 2.0, 1.0)):
        ch, sg = _state(K, n)
        with pytest.raises(K.KqftError):
            K.mfrg_flow(g, 1.0, T, li, lf, 1, 2, q, q, ch, sg, fo)
    ch, sg = _state(K, n)
    with pytest.raises(K.KqftError):
        K.mfrg_flow(g, 1.0, T, 2.0, 1.0, 0, 2, q, q, ch, sg)  # steps >= 1


def test_parquet_arguments():
    K = _K()
    g, q = K.Grid(5), K.Quad(11)
    for kw in ({"alpha": 0.0}, {"alpha": 1.5}, {"depth": 33}, {"depth": -1},
               {"reduce_alpha": True, "alpha_min": 0.9, "alpha": 0.5}, {"max_iterations": 0}):
        args = {"alpha": 0.5, "max_iterations": 2}
        args.update(kw)
        if args["max_iterations"] == 0:
            with pytest.raises((K.KqftError, ValueError)):
                K.parquet_solve(g, 1.0, D, T, q, q, **args)
            continue
        with pytest.raises(K.KqftError):
            K.parquet_solve(g, 1.0, D, T, q, q, **args)
    with pytest.raises(K.KqftError):  # Hartree quadrature must be valid
        K.parquet_solve(g, 1.0, D, T, q, q, max_iterations=1, eps_d=-0.3, q_hartree=K.Quad(0, 1, 0.0, 1.0))


def test_hartree_loop_propagator_and_adaptive_arguments():
    K = _K()
    n = 5
    qh = K.Quad(101, 1, 0.0, 1.0)
    with pytest.raises(K.KqftError):
        K.hartree(-1.0, 0.0, K.Propagator(D, T), qh)                  # U >= 0
    with pytest.raises(K.KqftError):
        K.hartree(1.0, 0.0, K.Propagator(D, T), qh, tol=0.0)          # tol > 0
    with pytest.raises(K.KqftError):
        K.hartree(1.0, 0.0, K.Propagator(D, T, reg=K.REG_U, lam=0.5), qh)
    V = K.Vertex(K.Grid(n), 1.0)
    s = torch.zeros(n, dtype=torch.complex128, device="cuda")
    with pytest.raises(K.KqftError):  # G Sigma_dot G line without Sigma_dot
        K.loop(V, K.Propagator(D, T), K.Quad(11), K.LINE_GSG)
    with pytest.raises(K.KqftError):  # Sigma_dot needs both components
        K.loop(V, K.Propagator(D, T, sigma_grid=K.Grid(n), dSigR=s), K.Quad(11), K.LINE_S)
    with pytest.raises(K.KqftError):  # the frequency regulator needs lam > 0
        K.loop(V, K.Propagator(D, T, reg=K.REG_NU, lam=0.0), K.Quad(11), K.LINE_S)
    with pytest.raises(K.KqftError):  # adaptive bubble: finite map only
        K.bubble_adaptive(0, V, V, K.Propagator(D, T), K.Quad(11, 1, 0.0, 1.0))
    with pytest.raises(K.KqftError):  # eps > 0
        K.bubble_adaptive(0, V, V, K.Propagator(D, T), K.Quad(11), eps=0.0)
    dout = K.alloc_channel(n)
    with pytest.raises(K.KqftError):  # adjoints take the plain Delta-regulated propagator
        K.bubble_adjoint(0, V, V, K.Propagator(D, T, reg=K.REG_U, lam=0.5), K.Quad(11), dout)


def test_asymmetric_flow_level_flow_and_chi_arguments():
    K = _K()
    n = 5
    g, q = K.Grid(n), K.Quad(11)
    ch, sg = _state(K, n)
    with pytest.raises(K.KqftError):  # the level must be finite
        K.mfrg_flow(g, 1.0, T, 2.0, 1.0, 1, 1, q, q, ch, sg, K.FlowOptions(eps_d=float("nan")))
    with pytest.raises(K.KqftError):
        K.mfrg_flow(g, 1.0, T, 2.0, 1.0, 1, 1, q, q, ch, sg, K.FlowOptions(eps_d=0.1, sigma_inf=float("inf")))
    V = K.Vertex(g, 1.0)
    with pytest.raises(K.KqftError):  # a non-finite level flow
        K.loop(V, K.Propagator(D, T, deps=float("nan")), q, K.LINE_S)
    with pytest.raises(K.KqftError):  # adjoints take no level flow
        K.bubble_adjoint(0, V, V, K.Propagator(D, T, deps=0.1), q, K.alloc_channel(n))
    with pytest.raises(K.KqftError):  # the Hartree term takes no level flow
        K.hartree(1.0, 0.0, K.Propagator(D, T, deps=0.1), K.Quad(101, 1, 0.0, 1.0))
    with pytest.raises(K.KqftError):  # channel 0..2
        K.chi(3, V, K.Propagator(D, T), q)
    with pytest.raises(K.KqftError):  # chi indexes the double sum in 32 bits
        K.chi(1, V, K.Propagator(D, T), K.Quad(46341))


def test_grid_size_limit():
    """A grid of more than 600 points is rejected (table records are indexed in 32 bits); the
    vertex's class arrays are never touched, so a tiny placeholder vertex suffices."""
    K = _K()
    g = K.Grid(601)
    V = K.Vertex(g, 1.0)  # bare vertex: no class arrays
    with pytest.raises(K.KqftError):
        K.chi(0, V, K.Propagator(D, T), K.Quad(11))
    with pytest.raises(K.KqftError):
        K.sde(V, K.Propagator(D, T), K.Quad(11), K.Quad(11))
