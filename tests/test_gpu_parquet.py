"""Parquet iteration and solver (Sec. parquet solver) on the GPU against the oracle.

One iteration -- the symmetrized Bethe-Salpeter equations of all three channels and the
Schwinger-Dyson self-energy, with a dynamic self-energy in the propagator -- agrees with the
oracle to 1e-12 on an arbitrary state; the solver (PT2 start, linear mixing) agrees with
the oracle's solver iterate by iterate.  At N = 51 the split-FP32 solver tracks the FP64
one and the time per iteration is reported.
"""
import time

import numpy as np
import pytest
import torch

import oracle as O
from workload import random_channel

pytestmark = pytest.mark.gpu

CL = ("K1", "K2", "K2p", "K3")
D, T, U = 1.0, 0.1, 1.0


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def test_parquet_iteration_matches_oracle():
    K = _K()
    n, nq = 11, 31
    chans = [random_channel(n, s, 0.1) for s in (3, 4, 5)]
    ov = O.Vertex(O.Grid(n), U, [O.Channel(1.0, *[c[x] for x in CL]) for c in chans])
    kv = K.Vertex(K.Grid(n), U, [K.Channel(1.0, *[to_dev(c[x]) for x in CL]) for c in chans])
    # a dynamic self-energy of the right analytic structure: the SDE of the same vertex
    sig0 = O.sde(ov, O.Prop(D, T), O.Quad(nq), O.Quad(nq))
    op = O.sigma_prop(O.Grid(n), D, T, sig0)
    kp = K.Propagator(D, T, sigma_grid=K.Grid(n), SigR=to_dev(sig0[:, 1]), SigK=to_dev(sig0[:, 0]))
    ref, rsig = O.parquet_iteration(ov, op, O.Quad(nq), O.Quad(nq))
    out, sig = K.parquet_iteration(kv, kp, K.Quad(nq), K.Quad(nq))
    torch.cuda.synchronize()
    for r in range(3):
        for x in CL:
            a, b = getattr(out[r], x).cpu().numpy(), getattr(ref[r], x)
            assert np.abs(a - b).max() < 1e-12 * np.abs(b).max(), (r, x)
    s = sig.cpu().numpy()
    assert np.abs(s - rsig).max() < 1e-12 * np.abs(rsig).max()


def test_parquet_solver_matches_oracle_iterates():
    K = _K()
    n, nq, iters = 9, 31, 6
    ochans, osig, ores = O.parquet_solve(O.Grid(n), U, D, T, O.Quad(nq), O.Quad(nq), alpha=0.5, iterations=iters)
    chans, sig, res = K.parquet_solve(K.Grid(n), U, D, T, K.Quad(nq), K.Quad(nq), alpha=0.5, max_iterations=iters)
    torch.cuda.synchronize()
    assert len(res) == iters
    assert np.allclose(res, ores, rtol=1e-9, atol=0)
    for r in range(3):
        for x in CL:
            a, b = getattr(chans[r], x).cpu().numpy(), getattr(ochans[r], x)
            assert np.abs(a - b).max() < 1e-11 * np.abs(b).max(), (r, x)
    assert np.abs(sig.cpu().numpy() - osig).max() < 1e-11 * np.abs(osig).max()


@pytest.mark.parametrize("U_,alpha,depth,reduce", [(1.0, 0.5, 3, False), (3.0, 1.0, 0, True), (3.0, 1.0, 2, True)])
def test_parquet_solver_anderson_and_reduction_match_oracle(U_, alpha, depth, reduce):
    """Anderson acceleration (normal equations on the device inner products) and the automatic
    reduction of the mixing factor: residuals and final state as the oracle's, n = 9."""
    K = _K()
    n, nq, iters = 9, 31, 8
    ochans, osig, ores = O.parquet_solve(O.Grid(n), U_, D, T, O.Quad(nq), O.Quad(nq), alpha=alpha, iterations=iters,
                                         depth=depth, reduce_alpha=reduce)
    chans, sig, res = K.parquet_solve(K.Grid(n), U_, D, T, K.Quad(nq), K.Quad(nq), alpha=alpha,
                                      max_iterations=iters, depth=depth, reduce_alpha=reduce)
    torch.cuda.synchronize()
    print(f"U={U_} alpha={alpha} depth={depth} reduce={reduce}: residuals {['%.2e' % x for x in res]}", flush=True)
    assert len(res) == iters
    assert np.allclose(res, ores, rtol=1e-8, atol=0)
    for r in range(3):
        for x in CL:
            a, b = getattr(chans[r], x).cpu().numpy(), getattr(ochans[r], x)
            assert np.abs(a - b).max() < 1e-9 * np.abs(b).max(), (r, x)
    assert np.abs(sig.cpu().numpy() - osig).max() < 1e-9 * np.abs(osig).max()


@pytest.mark.parametrize("eps_d", [None, -0.3])
def test_parquet_solver_with_the_mean_of_the_sde_forms_matches_oracle(eps_d):
    """sde_forms = 3: the self-energy as the mean of the SDE's a-, p- and t-forms (the oracle
    evaluates all three, the device (2 Sigma_a + Sigma_p) / 3 for the crossing-symmetric states);
    residuals and final state as the oracle's, at particle-hole symmetry and in the asymmetric
    model (whose states stay crossing symmetric too)."""
    K = _K()
    n, nq, iters = 9, 31, 6
    qh = (4001, 1, 0.0, 1.0)
    ow = {} if eps_d is None else {"eps_d": eps_d, "q_hartree": O.Quad(*qh), "hartree_tol": 1e-13}
    kw = {} if eps_d is None else {"eps_d": eps_d, "q_hartree": K.Quad(*qh), "hartree_tol": 1e-13}
    tol = 1e-11 if eps_d is None else 1e-9
    ores = O.parquet_solve(O.Grid(n), U, D, T, O.Quad(nq), O.Quad(nq), alpha=0.5, iterations=iters, sde_forms=3, **ow)
    kres = K.parquet_solve(K.Grid(n), U, D, T, K.Quad(nq), K.Quad(nq), alpha=0.5, max_iterations=iters, sde_forms=3,
                           **kw)
    torch.cuda.synchronize()
    ochans, osig, ors = ores[:3]
    chans, sig, res = kres[:3]
    print(f"eps_d={eps_d}: residuals {['%.2e' % x for x in res]}", flush=True)
    assert len(res) == iters
    assert np.allclose(res, ors, rtol=100 * tol, atol=0)
    for r in range(3):
        for x in CL:
            a, b = getattr(chans[r], x).cpu().numpy(), getattr(ochans[r], x)
            assert np.abs(a - b).max() < tol * np.abs(b).max(), (r, x)
    assert np.abs(sig.cpu().numpy() - osig).max() < tol * np.abs(osig).max()
    if eps_d is not None:
        assert abs(kres[3] - ores[3]) < 1e-10
    # the a-form alone gives another self-energy: the option reaches the device
    sig1 = K.parquet_solve(K.Grid(n), U, D, T, K.Quad(nq), K.Quad(nq), alpha=0.5, max_iterations=iters, **kw)[1]
    assert float((sig1 - sig).abs().max()) > 1e-6 * float(sig.abs().max())
    with pytest.raises(K.KqftError):
        K.parquet_solve(K.Grid(n), U, D, T, K.Quad(nq), K.Quad(nq), max_iterations=1, sde_forms=2)


def test_parquet_solver_n51_anderson_converges_faster():
    """N = 51, N_q = 501, U = 1: twelve iterations with Anderson depth 4 against linear mixing
    (split-FP32 bubbles); the accelerated residual ends an order of magnitude lower."""
    K = _K()
    n, nq, iters = 51, 501, 12
    g, q = K.Grid(n), K.Quad(nq)
    out = {}
    for depth in (0, 4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, res = K.parquet_solve(g, U, D, T, q, q, alpha=0.5, max_iterations=iters, precision=K.SPLIT_FP32,
                                    depth=depth)
        torch.cuda.synchronize()
        out[depth] = (res, (time.perf_counter() - t0) / iters)
    print(f"parquet n={n}: linear mixing {out[0][1] * 1e3:.1f} ms/iteration, residual {out[0][0][-1]:.2e}; "
          f"Anderson m=4 {out[4][1] * 1e3:.1f} ms/iteration, residual {out[4][0][-1]:.2e}", flush=True)
    assert out[4][0][-1] < 0.1 * out[0][0][-1]


def test_parquet_solver_n51_split_tracks_fp64():
    K = _K()
    n, nq, iters = 51, 501, 12
    g, q = K.Grid(n), K.Quad(nq)
    times = {}
    outs = {}
    for name, prec in (("fp64", K.FP64), ("split", K.SPLIT_FP32)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs[name] = K.parquet_solve(g, U, D, T, q, q, alpha=0.5, max_iterations=iters, precision=prec)
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / iters
    (c64, s64, r64), (c32, s32, r32) = outs["fp64"], outs["split"]
    print(f"parquet n={n} nq={nq}: {times['fp64'] * 1e3:.1f} ms/iteration FP64, {times['split'] * 1e3:.1f} split; "
          f"residuals {r64[0]:.2e} -> {r64[-1]:.2e}", flush=True)
    assert r64[-1] < 0.05 * r64[2]  # contracting
    worst = 0.0
    for r in range(3):
        for x in CL:
            a, b = getattr(c32[r], x), getattr(c64[r], x)
            worst = max(worst, float((a - b).abs().max() / b.abs().max()))
    worst = max(worst, float((s32 - s64).abs().max() / s64.abs().max()))
    print(f"split vs fp64 after {iters} iterations: {worst:.2e}", flush=True)
    assert worst < 1e-5


def test_parquet_iteration_time_n101():
    """Three split-FP32 solver iterations at N = 101, Nq = 1001 (6 bubbles of 1.08 TFLOP each
    plus the self-energy per iteration); the residual decreases."""
    K = _K()
    n, nq, iters = 101, 1001, 3
    g, q = K.Grid(n), K.Quad(nq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chans, sig, res = K.parquet_solve(g, U, D, T, q, q, alpha=0.5, max_iterations=iters, precision=K.SPLIT_FP32)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    flop = 6 * 2.0 * n * 8.0 * (4 * n + 4) * 4.0 * nq * (4 * n + 4)
    print(f"parquet n={n}: {dt * 1e3:.1f} ms/iteration, {flop / dt / 1e12:.1f} TFLOP/s in the bubbles' "
          f"algorithmic count; residuals {['%.2e' % x for x in res]}", flush=True)
    assert len(res) == iters and res[2] < res[1] < res[0]
