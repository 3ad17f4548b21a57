"""kqft_regrid on the GPU against the oracle: random classes and a self-energy carried between
tangent and algebraic grids (also beyond the source extent), and a hybridization flow whose
grid is rescaled with the flow parameter between two segments (Sec. Frequency grids)."""
import numpy as np
import pytest
import torch

import oracle as O
from workload import random_channel

pytestmark = pytest.mark.gpu

CL = ("K1", "K2", "K2p", "K3")
T = 0.1
EINVAL, ESHAPE = -1, -2  # KQFT_EINVAL, KQFT_ESHAPE


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _grids(K, n, L, a, mp):
    return O.Grid(n, L, a, mp), K.Grid(n, L, a, mp)


@pytest.mark.parametrize("src,dst", [((9, 20.0, 1.0, 0), (11, 15.0, 0.6, 1)), ((10, 20.0, 0.8, 1), (7, 25.0, 1.3, 0))])
def test_regrid_matches_oracle(src, dst):
    K = _K()
    os_, ks = _grids(K, *src)
    od, kd = _grids(K, *dst)
    raw = [random_channel(src[0], 60 + r) for r in range(3)]
    sig = np.random.default_rng(2).standard_normal((src[0], 4)) * (1 + 0.5j)
    ref, rsig = O.regrid(os_, od, [O.Channel(0.5 + r, **c) for r, c in enumerate(raw)], sig)
    chans = [K.Channel(0.5 + r, *[to_dev(c[x]) for x in CL]) for r, c in enumerate(raw)]
    new, ksig = K.regrid(ks, kd, chans, to_dev(sig))
    torch.cuda.synchronize()
    for r in range(3):
        assert new[r].coef == 0.5 + r
        for x in CL:
            a, b = getattr(new[r], x).cpu().numpy(), getattr(ref[r], x)
            assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max(), (r, x)
    assert np.abs(ksig.cpu().numpy() - rsig).max() <= 1e-13 * np.abs(rsig).max()


def test_flow_with_a_grid_rescaled_between_segments_matches_oracle():
    """Delta-flow 2 -> 1.5 on a grid of scale a = 2, regrid to a = 1.5, flow 1.5 -> 1 (RK4, three
    loops, Katanin), from the PT2 state: the scale follows the hybridization."""
    K = _K()
    n, nq, U, nl = 9, 31, 1.0, 3
    q = O.Quad(nq)
    g1, k1 = _grids(K, n, 20.0, 2.0, 0)
    g2, k2 = _grids(K, n, 20.0, 1.5, 0)
    chans, sig = O.pt2_state(g1, U, 2.0, T, q, q)
    och, osig, _ = O.mfrg_flow(g1, U, T, 2.0, 1.5, 1, nl, q, q, chans, sig, O.FlowOptions())
    och, osig = O.regrid(g1, g2, och, osig)
    och, osig, _ = O.mfrg_flow(g2, U, T, 1.5, 1.0, 1, nl, q, q, och, osig, O.FlowOptions())
    kch = [K.Channel(1.0, *[to_dev(getattr(c, x)) for x in CL]) for c in chans]
    ksig = to_dev(sig)
    K.mfrg_flow(k1, U, T, 2.0, 1.5, 1, nl, K.Quad(nq), K.Quad(nq), kch, ksig, K.FlowOptions())
    kch, ksig = K.regrid(k1, k2, kch, ksig)
    K.mfrg_flow(k2, U, T, 1.5, 1.0, 1, nl, K.Quad(nq), K.Quad(nq), kch, ksig, K.FlowOptions())
    torch.cuda.synchronize()
    for r in range(3):
        for x in CL:
            a, b = getattr(kch[r], x).cpu().numpy(), getattr(och[r], x)
            assert np.abs(a - b).max() <= 1e-10 * max(np.abs(b).max(), 1e-300), (r, x)
    assert np.abs(ksig.cpu().numpy() - osig).max() < 1e-10 * np.abs(osig).max()


def test_regrid_errors():
    K = _K()
    g = K.Grid(5)
    lib, C = K.lib(), K.C
    s = torch.zeros((5, 4), dtype=torch.complex128, device="cuda")
    gc = g.c()
    p = C.c_void_p(s.data_ptr())
    assert lib.kqft_regrid(K.ctx(), C.byref(gc), C.byref(gc), None, p, None, p, None) == EINVAL  # in place
    assert lib.kqft_regrid(K.ctx(), C.byref(gc), C.byref(gc), None, p, None, None, None) == EINVAL
    assert lib.kqft_regrid(K.ctx(), C.byref(gc), C.byref(gc), None, None, None, None, None) == EINVAL
    bad = K.Grid(1).c()
    t = torch.zeros((1, 4), dtype=torch.complex128, device="cuda")
    assert lib.kqft_regrid(K.ctx(), C.byref(gc), C.byref(bad), None, p, None, C.c_void_p(t.data_ptr()),
                           None) == ESHAPE
