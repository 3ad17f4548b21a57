"""torch.autograd Functions over the HIP bubble and Schwinger-Dyson entry points.

Forward calls kqft_bubble / kqft_sde / kqft_mloop_step; backward calls
kqft_bubble_adjoint / kqft_sde_adjoint / kqft_mloop_adjoint, which recompute the panels
and the multiloop insertions (no activation storage beyond the vertex tensors
themselves); forward-mode tangents of the insertions come from kqft_mloop_jvp.  This
module only marshals tensors: every sum of the method runs in the library.  Differentiable inputs: the class tensors of every
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
        channel, kind, grid, q, T, eps, coefsL, coefsR, precision, cmask = meta
        fl, fr = list(tensors[:12]), list(tensors[12:])
        L = _kvertex(grid, r0L, coefsL, fl)
        R = _kvertex(grid, r0R, coefsR, fr)
        P = K.Propagator(float(Delta), T, eps)
        out = K.bubble(channel, L, R, P, q, pi_kind=kind, precision=precision, class_mask=cmask)
        ctx.meta = meta
        ctx.save_for_backward(r0L, r0R, Delta, *tensors)
        return out.K1, out.K2, out.K2p, out.K3

    @staticmethod
    def backward(ctx, g1, g2, g2p, g3):
        channel, kind, grid, q, T, eps, coefsL, coefsR, _, cmask = ctx.meta
        # classes outside the mask are returned as constant zeros: their cotangents do not flow
        g1, g2, g2p, g3 = [g if (cmask & bit) else None
                           for g, bit in zip((g1, g2, g2p, g3), (K.K1, K.K2, K.K2P, K.K3))]
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
           eps: float = 0.0, kind: int = K.PI_GG, precision: int = K.FP64, class_mask: int = K.KALL) -> dict:
    """B_channel(left, right) as a dict of class tensors; classes outside class_mask are zero."""
    meta = (channel, kind, left.grid, q, T, eps, left.coefs, right.coefs, precision, class_mask)
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


class _MLoop(torch.autograd.Function):
    """Multiloop insertions of kqft_mloop_step; backward through kqft_mloop_adjoint, which
    recomputes the insertions order by order (only the vertex tensors are saved)."""

    @staticmethod
    def forward(ctx, meta, r0, Delta, *tensors):
        grid, q, T, eps, coefs, nloops, precision = meta
        V = _kvertex(grid, r0, coefs, list(tensors))
        out = K.mloop_step([V], [K.Propagator(float(Delta), T, eps)], [q], nloops, precision=precision)[0]
        ctx.meta = meta
        ctx.save_for_backward(r0, Delta, *tensors)
        return tuple(getattr(out[l][r], x) for l in range(nloops) for r in range(3) for x in K.CLASSES)

    @staticmethod
    def backward(ctx, *grads):
        grid, q, T, eps, coefs, nloops, _ = ctx.meta
        saved = ctx.saved_tensors
        r0, Delta = saved[:2]
        flat = list(saved[2:])
        V = _kvertex(grid, r0, coefs, flat)
        dgdot = [[None] * 3 for _ in range(nloops)]
        for l in range(nloops):
            for r in range(3):
                g4 = grads[4 * (3 * l + r): 4 * (3 * l + r) + 4]
                if any(g is not None for g in g4):
                    dgdot[l][r] = K.Channel(1.0, *[(g.contiguous() if g is not None else None) for g in g4])
        dG = _grads_like(flat, coefs)
        dscal = K.mloop_adjoint(V, K.Propagator(float(Delta), T, eps), q, nloops, dgdot, dgamma=dG).cpu()
        return (None, dscal[0], dscal[1], *_flat_grads(dG))


def mloop(gamma: TVertex, Delta: torch.Tensor, q: K.Quad, T: float, nloops: int, eps: float = 0.0,
          precision: int = K.FP64) -> list:
    """Multiloop insertions of the mfRG flow (Eqs. 1l-3l; Delta-flow single-scale propagator,
    no Katanin term) as a differentiable function of the vertex, r0 and Delta: out[l-1][r] is a
    dict of class tensors of the order-l insertion of channel r (left + right + centre)."""
    meta = (gamma.grid, q, T, eps, gamma.coefs, nloops, precision)
    outs = _MLoop.apply(meta, gamma.r0, Delta, *gamma.flat())
    return [[dict(zip(K.CLASSES, outs[4 * (3 * l + r): 4 * (3 * l + r) + 4])) for r in range(3)]
            for l in range(nloops)]


# ------------------------------------------------------------------ forward mode
# The bubble is bilinear in its two vertices, so at a fixed propagator its tangent along
# vertex tangents (dL, dR) is B(dL, R) + B(L, dR): two more bubbles.  A tangent vertex holds
# the tangent of r0 and of the class arrays (channels without tangent arrays carry none).

def bubble_jvp(channel: int, L: K.Vertex, dL: K.Vertex, R: K.Vertex, dR: K.Vertex, G: K.Propagator, q: K.Quad,
               kind: int = K.PI_GG, precision: int = K.FP64, class_mask: int = K.KALL):
    out = K.bubble(channel, L, R, G, q, pi_kind=kind, precision=precision, class_mask=class_mask)
    dout = K.bubble(channel, dL, R, G, q, pi_kind=kind, precision=precision, class_mask=class_mask)
    K.bubble(channel, L, dR, G, q, pi_kind=kind, precision=precision, class_mask=class_mask, out=dout, beta=1)
    return out, dout


def mloop_jvp(gamma: K.Vertex, dgamma: K.Vertex, G: K.Propagator, q: K.Quad, nloops: int,
              precision: int = K.FP64):
    """Multiloop insertions and their tangents along the vertex tangent dgamma at a fixed
    propagator (kqft_mloop_jvp).  Returns (out, dout), each out[l-1][r] a Channel."""
    return K.mloop_jvp(gamma, dgamma, G, q, nloops, precision=precision)
