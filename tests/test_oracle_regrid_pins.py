"""Pins of the oracle's regridding (the classes and the self-energy carried from one frequency
grid onto another by the interpolation every lookup uses, Sec. Interpolation routines; the
paper rescales its grids during hybridization flows, Sec. Frequency grids).

Onto the same grid it is the identity; onto another grid it reproduces exactly any function
that is multilinear in the source grid's auxiliary variables (here evaluated with numpy's
arctan, not through the oracle's grid code); points beyond the source extent read zero."""
import numpy as np

from oracle import oracle as O
from workload import random_channel

CL = ("K1", "K2", "K2p", "K3")


def test_regrid_onto_the_same_grid_is_the_identity():
    g = O.Grid(9, 20.0, 1.0)
    chans = [O.Channel(1.0, **random_channel(9, 40 + r)) for r in range(3)]
    sig = np.random.default_rng(1).standard_normal((9, 4)) + 0j
    new, s2 = O.regrid(g, g, chans, sig)
    for r in range(3):
        for x in CL:
            assert np.abs(getattr(new[r], x) - getattr(chans[r], x)).max() < 1e-15
    assert np.abs(s2 - sig).max() < 1e-15


def test_regrid_reproduces_multilinear_functions_of_the_source_auxiliary_variable():
    src = O.Grid(11, 20.0, 1.0)              # tangent: x(v) = atan(v/a)/atan(L/a)
    dst = O.Grid(8, 15.0, 0.6, 1)            # algebraic, inside the source extent
    x = lambda v: np.arctan(v / src.a) / np.arctan(src.L / src.a)
    xs, xd = x(src.nodes()), x(dst.nodes())
    rng = np.random.default_rng(3)
    c = rng.standard_normal((8, 2, 16)) + 1j * rng.standard_normal((8, 2, 16))

    def f3(a, b, d):  # multilinear in (a, b, d), one coefficient set per spin and component
        A, B, D = np.meshgrid(a, b, d, indexing="ij")
        terms = [np.ones_like(A), A, B, D, A * B, A * D, B * D, A * B * D]
        return np.einsum("tsk,tijl->sijlk", c, np.array(terms))

    K3 = f3(xs, xs, xs)
    K2 = f3(xs, xs, np.zeros(1))[:, :, :, 0]
    K1 = f3(xs, np.zeros(1), np.zeros(1))[:, :, 0, 0]
    chans = [O.Channel(0.5, K1, K2, K2.copy(), K3) for _ in range(3)]
    sig = (1.0 + 2.0j) + (0.5 - 1.5j) * np.tile(xs[:, None], (1, 4))
    new, s2 = O.regrid(src, dst, chans, sig)
    for r in range(3):
        assert new[r].coef == 0.5
        assert np.abs(new[r].K3 - f3(xd, xd, xd)).max() < 1e-12
        assert np.abs(new[r].K2 - f3(xd, xd, np.zeros(1))[:, :, :, 0]).max() < 1e-12
        assert np.abs(new[r].K2p - f3(xd, xd, np.zeros(1))[:, :, :, 0]).max() < 1e-12
        assert np.abs(new[r].K1 - f3(xd, np.zeros(1), np.zeros(1))[:, :, 0, 0]).max() < 1e-12
    assert np.abs(s2 - ((1.0 + 2.0j) + (0.5 - 1.5j) * xd[:, None])).max() < 1e-13


def test_regrid_beyond_the_source_extent_reads_zero():
    src, dst = O.Grid(7, 5.0, 1.0), O.Grid(9, 20.0, 1.0)
    chans = [O.Channel(1.0, **random_channel(7, 50 + r)) for r in range(3)]
    sig = np.ones((7, 4), complex)
    new, s2 = O.regrid(src, dst, chans, sig)
    out = np.abs(dst.nodes()) > 5.0 * (1 + 1e-9)
    assert out.any() and np.all(s2[out] == 0) and np.all(s2[~out] == 1)
    for r in range(3):
        assert np.all(new[r].K1[:, out] == 0) and np.all(new[r].K3[:, :, :, out] == 0)
        assert np.all(new[r].K2[:, out, :] == 0)
