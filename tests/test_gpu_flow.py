"""Vertex loop and multiloop fRG flow (Sec. loop, Sec. mfRG) on the GPU against the oracle.

kqft_loop evaluates the loop of a full vertex (all three channels at their own parameters)
with G or S; kqft_mfrg_flow integrates the Delta-flow with the classical Runge-Kutta rule
(multiloop vertex insertions, one-loop self-energy flow) and agrees with the oracle's flow
step by step at FP64 rounding.  At N = 51 the flow is timed and the split-FP32 run tracks
the FP64 one.
"""
import time

import numpy as np
import pytest
import torch

import oracle as O
from workload import random_channel

pytestmark = pytest.mark.gpu

CL = ("K1", "K2", "K2p", "K3")
T = 0.1


def _K():
    from paper_2405_20996_amd import kqft as K
    return K


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("kind", [0, 1])
def test_vertex_loop_matches_oracle(kind):
    K = _K()
    n, nq = 13, 41
    coefs = (1.0, 0.8, 1.2)
    chans = [random_channel(n, s, 0.2) for s in (7, 8, 9)]
    ov = O.Vertex(O.Grid(n), 0.7, [O.Channel(c, *[ch[x] for x in CL]) for c, ch in zip(coefs, chans)])
    kv = K.Vertex(K.Grid(n), 0.7, [K.Channel(c, *[to_dev(ch[x]) for x in CL]) for c, ch in zip(coefs, chans)])
    sg = O.sde(ov, O.Prop(1.0, T), O.Quad(nq), O.Quad(nq))
    op = O.sigma_prop(O.Grid(n), 1.0, T, sg)
    kp = K.Propagator(1.0, T, sigma_grid=K.Grid(n), SigR=to_dev(sg[:, 1]), SigK=to_dev(sg[:, 0]))
    ref = O.loop(ov, op, O.Quad(nq), kind)
    out = K.loop(kv, kp, K.Quad(nq), kind).cpu().numpy()
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()


def gpu_state(K, chans, sig):
    return ([K.Channel(1.0, *[to_dev(getattr(c, x)) for x in CL]) for c in chans], to_dev(sig))


def test_mfrg_flow_matches_oracle():
    K = _K()
    n, nq, U, steps, nl = 9, 31, 1.0, 2, 3
    g, q = O.Grid(n), O.Quad(nq)
    chans, sig = O.pt2_state(g, U, 2.0, T, q, q)
    rch, rsig = O.mfrg_flow(g, U, T, 2.0, 1.0, steps, nl, q, q, chans, sig)
    kch, ksig = gpu_state(K, chans, sig)
    K.mfrg_flow(K.Grid(n), U, T, 2.0, 1.0, steps, nl, K.Quad(nq), K.Quad(nq), kch, ksig)
    torch.cuda.synchronize()
    for r in range(3):
        for x in CL:
            a, b = getattr(kch[r], x).cpu().numpy(), getattr(rch[r], x)
            assert np.abs(a - b).max() < 1e-11 * np.abs(b).max(), (r, x)
    assert np.abs(ksig.cpu().numpy() - rsig).max() < 1e-11 * np.abs(rsig).max()


def test_mfrg_flow_n51_timing_and_split():
    K = _K()
    n, nq, U, steps, nl = 51, 501, 1.0, 2, 3
    g, q = O.Grid(n), O.Quad(nq)
    chans, sig = O.pt2_state(g, U, 2.0, T, q, q)
    res, times = {}, {}
    for name, prec in (("fp64", K.FP64), ("split", K.SPLIT_FP32)):
        kch, ksig = gpu_state(K, chans, sig)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K.mfrg_flow(K.Grid(n), U, T, 2.0, 1.0, steps, nl, K.Quad(nq), K.Quad(nq), kch, ksig, precision=prec)
        torch.cuda.synchronize()
        times[name] = time.perf_counter() - t0
        res[name] = (kch, ksig)
    worst = 0.0
    for r in range(3):
        for x in CL:
            a, b = getattr(res["split"][0][r], x), getattr(res["fp64"][0][r], x)
            worst = max(worst, float((a - b).abs().max() / b.abs().max()))
    worst = max(worst, float((res["split"][1] - res["fp64"][1]).abs().max() / res["fp64"][1].abs().max()))
    print(f"mfRG flow n={n} nq={nq} l<={nl}, {steps} RK4 steps ({4 * steps} right-hand sides of "
          f"{3 + 6 + 9 * (nl - 2)} bubbles): {times['fp64']:.2f} s FP64, {times['split']:.2f} s split; "
          f"split vs fp64 {worst:.2e}", flush=True)
    assert worst < 1e-5
