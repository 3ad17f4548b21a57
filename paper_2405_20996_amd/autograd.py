"""torch.autograd Functions over the HIP bubble and Schwinger-Dyson entry points.

Forward calls kqft_bubble / kqft_sde; backward calls kqft_bubble_adjoint /
kqft_sde_adjoint, which recompute the panels (no activation storage beyond the
vertex tensors themselves).  Differentiable inputs: the class tensors of every
channel (complex128), the bare-vertex strength r0 and the hybridization Delta
(0-dim float64 tensors on the CPU).  Gradients follow PyTorch's convention for
complex tensors (dL/dRe z + i dL/dIm z).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import torch

from . import kqft as K


@dataclass
class TVertex:
    """Vertex with differentiable parts: r0 (0-dim tensor) and per-channel class tensors."""
    grid: K.Grid
    r0: torch.Tensor
    coefs: tuple = (1.0, 1.0, 1.0)
    ch: list = field(default_factory=lambda: [dict(), dict(), dict()])  # ch[r][class] -> tensor

    def flat(self) -> list:
        return [self.ch[r].get(c) for r in range(3) for c in K.CLASSES]


def _kvertex(grid, r0, coefs, flat):
    chans = []
    for r in range(3):
        t = flat[4 * r: 4 * r + 4]
        has = any(x is not None for x in t)
        chans.append(K.Channel(coefs[r] if has else 0.0, *[(x.detach() if x is not None else None) for x in t]))
    return K.Vertex(grid, float(r0), chans)


def _grads_like(flat, coefs):
    out = []
    for r in range(3):
        t = flat[4 * r: 4 * r + 4]
        if all(x is None for x in t):
            out.append(None)
            continue
        out.append(K.Channel(1.0, *[(torch.zeros_like(x) if x is not None else None) for x in t]))
    return out


def _flat_grads(chans):
    res = []
    for c in chans:
        for name in K.CLASSES:
            res.append(None if c is None else getattr(c, name))
    return res


class _Bubble(torch.autograd.Function):
    @staticmethod
    def forward(ctx, meta, r0L, r0R, Delta, *tensors):
        channel, kind, grid, q, T, eps, coefsL, coefsR, precision = meta
        fl, fr = list(tensors[:12]), list(tensors[12:])
        L = _kvertex(grid, r0L, coefsL, fl)
        R = _kvertex(grid, r0R, coefsR, fr)
        P = K.Propagator(float(Delta), T, eps)
        out = K.bubble(channel, L, R, P, q, pi_kind=kind, precision=precision)
        ctx.meta = meta
        ctx.save_for_backward(r0L, r0R, Delta, *tensors)
        return out.K1, out.K2, out.K2p, out.K3

    @staticmethod
    def backward(ctx, g1, g2, g2p, g3):
        channel, kind, grid, q, T, eps, coefsL, coefsR, _ = ctx.meta
        saved = ctx.saved_tensors
        r0L, r0R, Delta = saved[:3]
        fl, fr = list(saved[3:15]), list(saved[15:27])
        L = _kvertex(grid, r0L, coefsL, fl)
        R = _kvertex(grid, r0R, coefsR, fr)
        P = K.Propagator(float(Delta), T, eps)
        n = grid.n
        dout = K.Channel(1.0, *[(g.contiguous() if g is not None else torch.zeros(K.class_shape(c, n),
                                                                                   dtype=torch.complex128,
                                                                                   device="cuda"))
                                for g, c in zip((g1, g2, g2p, g3), K.CLASSES)])
        dL = _grads_like(fl, coefsL)
        dR = _grads_like(fr, coefsR)
        dscal = K.bubble_adjoint(channel, L, R, P, q, dout, pi_kind=kind, dleft=dL, dright=dR).cpu()
        return (None, dscal[0], dscal[1], dscal[2], *_flat_grads(dL), *_flat_grads(dR))


def bubble(channel: int, left: TVertex, right: TVertex, Delta: torch.Tensor, q: K.Quad, T: float,
           eps: float = 0.0, kind: int = K.PI_GG, precision: int = K.FP64) -> dict:
    meta = (channel, kind, left.grid, q, T, eps, left.coefs, right.coefs, precision)
    outs = _Bubble.apply(meta, left.r0, right.r0, Delta, *left.flat(), *right.flat())
    return dict(zip(K.CLASSES, outs))


class _SDE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, meta, r0, Delta, *tensors):
        grid, qb, ql, T, eps, coefs = meta
        V = _kvertex(grid, r0, coefs, list(tensors))
        sigma, _ = K.sde(V, K.Propagator(float(Delta), T, eps), qb, ql, with_chi=False)
        ctx.meta = meta
        ctx.save_for_backward(r0, Delta, *tensors)
        return sigma

    @staticmethod
    def backward(ctx, dsigma):
        grid, qb, ql, T, eps, coefs = ctx.meta
        saved = ctx.saved_tensors
        r0, Delta = saved[:2]
        flat = list(saved[2:])
        V = _kvertex(grid, r0, coefs, flat)
        dG = _grads_like(flat, coefs)
        dscal = K.sde_adjoint(V, K.Propagator(float(Delta), T, eps), qb, ql, dsigma.contiguous(), dgamma=dG).cpu()
        return (None, dscal[0], dscal[1], *_flat_grads(dG))


def sde(gamma: TVertex, Delta: torch.Tensor, q_bubble: K.Quad, q_loop: K.Quad, T: float, eps: float = 0.0):
    """Dynamic self-energy [n][4] from the Schwinger-Dyson equation (a-channel form)."""
    meta = (gamma.grid, q_bubble, q_loop, T, eps, gamma.coefs)
    return _SDE.apply(meta, gamma.r0, Delta, *gamma.flat())
