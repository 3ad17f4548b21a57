"""Finite-temperature Matsubara formalism (MF) of the bubble, loop and Schwinger-Dyson equation.

TEST INFRASTRUCTURE ONLY, like the rest of this package.  The paper carries its diagrammatic
functions over to discrete Matsubara sums in the finite-T MF (Sec. Introduction: flexibility,
Sec. Vectorization: the Matsubara sums as matrix products); the formulas are the Keldysh ones
with the Keldysh structure removed, written here directly:

  frequencies   nu_n = (2n + 1) pi T (fermionic), Omega_m = 2 m pi T (bosonic);
  legs (integer parametrisation, every leg frequency fermionic):
      a: n2 = n, n1' = n + m, n2' = n', n1 = n' + m        (omega = nu1' - nu2)
      p: n1' = n, n2' = m - n - 1, n1 = n', n2 = m - n' - 1  (omega = nu1' + nu2')
      t: n2 = n, n2' = n + m, n1' = n', n1 = n' + m        (omega = nu2' - nu2)
  classes       K1[s][m], K2[s][m][n], K2'[s][m][n'], K3[s][m][n][n'] on m in [-M, M],
                n, n' in [-N, N), spin s = X (up-down|up-down), Y (up-down|down-up); zero outside;
  bare vertex   X0 = -U, Y0 = +U;
  propagator    G(i nu_n) = 1 / (i nu_n + i Delta sgn(nu_n) - Sigma(n)) (level 0: particle-hole
                symmetry with U/2 absorbed; Sigma given on [-Ns, Ns), zero outside);
  bubbles       B_r(L, R)(m; n, n') = pref_r T sum_{n''} L(m; n, n'') Pi_r(m, n'') R(m; n'', n')
                (spin sums below), Pi_a = Pi_t = G(n'' + m) G(n''), Pi_p = G(n'') G(m - n'' - 1),
                pref_r = +1, 1/2, -1; the sum over the window |2n'' + 1 + s m| <= 2 Nq - 1,
                s = +1 (a, t) or -1 (p), symmetric about the bubble's centre;
  asymptotic classes as in the Keldysh formalism: L^inf = Gamma_0 + K1 + K2' (own channel at
                (m, n'')), R^inf = Gamma_0 + K1 + K2, K3 = (L - L^inf) Pi (R - R^inf) etc.;
  loop          L(Gamma, G)(n) = T sum_{n'} [2 X + Y](legs n, n' | n, n') G(n'), window
                |2n' + 1| <= 2 Nl - 1;  SDE  Sigma = -1/2 L(B_a(Gamma_0, Gamma), G).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

CLASSES = ("K1", "K2", "K2p", "K3")


def nu(n, T: float):
    return (2.0 * np.asarray(n) + 1.0) * np.pi * T


def om(m, T: float):
    return 2.0 * np.asarray(m) * np.pi * T


@dataclass
class MGrid:
    """Bosonic box m in [-M, M], fermionic box n in [-N, N), temperature T."""
    M: int
    N: int
    T: float

    def shapes(self):
        nb, nf = 2 * self.M + 1, 2 * self.N
        return {"K1": (2, nb), "K2": (2, nb, nf), "K2p": (2, nb, nf), "K3": (2, nb, nf, nf)}


@dataclass
class MChannel:
    coef: float = 1.0
    K1: Optional[np.ndarray] = None
    K2: Optional[np.ndarray] = None
    K2p: Optional[np.ndarray] = None
    K3: Optional[np.ndarray] = None


@dataclass
class MVertex:
    grid: MGrid
    U: float = 0.0
    ch: list = field(default_factory=lambda: [MChannel(0.0), MChannel(0.0), MChannel(0.0)])


def legs_of(r: int, m, n, npr):
    """Leg indices (n1', n2', n1, n2) of channel r's parameters (m, n, n')."""
    m, n, npr = np.asarray(m), np.asarray(n), np.asarray(npr)
    if r == 0:
        return n + m, npr, npr + m, n
    if r == 1:
        return n, m - n - 1, npr, m - npr - 1
    return npr, n + m, npr + m, n


def params_of(r: int, n1p, n2p, n1, n2):
    """Channel r's parameters (m, n, n') of the legs (inverse of legs_of on conserving legs)."""
    if r == 0:
        return n1p - n2, n2, n2p
    if r == 1:
        return n1p + n2p + 1, n1p, n1
    return n2p - n2, n2, n1p


def _lookup(arr: Optional[np.ndarray], grid: MGrid, idx):
    """arr[s][m + M][n + N]... at integer indices (per spin), zero outside the box or when absent."""
    shape = np.broadcast(*idx).shape
    out = np.zeros((2,) + shape, dtype=np.complex128)
    if arr is None:
        return out
    offs = [grid.M] + [grid.N] * (len(idx) - 1)
    lims = [2 * grid.M + 1] + [2 * grid.N] * (len(idx) - 1)
    ii = [np.broadcast_to(np.asarray(x) + o, shape) for x, o in zip(idx, offs)]
    ok = np.ones(shape, dtype=bool)
    for x, lim in zip(ii, lims):
        ok &= (x >= 0) & (x < lim)
    safe = [np.where(ok, x, 0) for x in ii]
    for s in range(2):
        out[s] = np.where(ok, arr[s][tuple(safe)], 0.0)
    return out


def channel_value(c: MChannel, grid: MGrid, m, n, npr, parts=CLASSES):
    """Sum of the selected classes of one channel at its own parameters: [2, ...] (X, Y)."""
    m, n, npr = np.broadcast_arrays(np.asarray(m), np.asarray(n), np.asarray(npr))
    v = np.zeros((2,) + m.shape, dtype=np.complex128)
    if "K1" in parts:
        v = v + _lookup(c.K1, grid, (m,))
    if "K2" in parts:
        v = v + _lookup(c.K2, grid, (m, n))
    if "K2p" in parts:
        v = v + _lookup(c.K2p, grid, (m, npr))
    if "K3" in parts:
        v = v + _lookup(c.K3, grid, (m, n, npr))
    return c.coef * np.asarray(v)


def vertex_eval(V: MVertex, r: int, m, n, npr):
    """The full vertex Gamma_0 + sum_r' coef gamma_r' at channel r's parameters: [2, ...] (X, Y);
    every channel is read at its own parameters of the same legs (exact indices, no
    interpolation)."""
    legs = legs_of(r, m, n, npr)
    shape = np.broadcast(*legs).shape
    out = np.zeros((2,) + shape, dtype=np.complex128)
    out[0] += -V.U
    out[1] += V.U
    for r2 in range(3):
        c = V.ch[r2]
        if c.coef == 0.0:
            continue
        m2, n2, np2 = params_of(r2, *legs)
        out += channel_value(c, V.grid, m2, n2, np2)
    return out


def vertex_legs(V: MVertex, spins, legs):
    """Gamma_{s1' s2' | s1 s2}(n1', n2' | n1, n2) = X d(s1', s1) d(s2', s2) + Y d(s1', s2) d(s2', s1)
    (SU(2), the spin structure of every channel), read through channel a's parameters."""
    n1p, n2p, n1, n2 = [np.asarray(x) for x in legs]
    s1p, s2p, s1, s2 = [np.asarray(x) for x in spins]
    XY = vertex_eval(V, 0, *params_of(0, n1p, n2p, n1, n2))
    return XY[0] * ((s1p == s1) & (s2p == s2)) + XY[1] * ((s1p == s2) & (s2p == s1))


def _on_box(arr: Optional[np.ndarray], n: np.ndarray) -> np.ndarray:
    """arr[n + Ns] on n in [-Ns, Ns) (len(arr) = 2 Ns), zero elsewhere or when absent."""
    if arr is None:
        return np.zeros(n.shape, dtype=np.complex128)
    Ns = len(arr) // 2
    ok = (n >= -Ns) & (n < Ns)
    return np.where(ok, arr[np.where(ok, n + Ns, 0)], 0.0)


@dataclass
class MProp:
    """G(i nu_n) = 1/(i nu_n + i Delta sgn(nu_n) - Sigma(n)), Sigma on n in [-Ns, Ns) or none.
    The flow parameter is Delta (reg 0, hybridization flow; S = dG/dDelta at fixed Sigma =
    -i sgn(nu) G^2) or lam (reg 1, interaction flow, Sec. Flow schemes: G_0 -> lam G_0, so
    G = 1/(G_0^-1/lam - Sigma) and S = dG/dlam at fixed Sigma = G G_0^-1 G / lam^2), plus
    G Sigma_dot G with the optional dsigma (Katanin substitution)."""
    Delta: float
    T: float
    sigma: Optional[np.ndarray] = None
    dsigma: Optional[np.ndarray] = None
    reg: int = 0
    lam: float = 1.0

    def g0inv(self, n):
        v = nu(np.asarray(n), self.T)
        return 1j * v + 1j * self.Delta * np.sign(v)

    def __call__(self, n):
        n = np.asarray(n)
        scale = 1.0 / self.lam if self.reg == 1 else 1.0
        return 1.0 / (self.g0inv(n) * scale - _on_box(self.sigma, n))

    def line(self, n, kind: int = 0):
        """kind 0: G; 1: S (+ G Sigma_dot G with dsigma); 2: G Sigma_dot G."""
        n = np.asarray(n)
        g = self(n)
        if kind == 0:
            return g
        gsg = g * _on_box(self.dsigma, n) * g
        if kind == 2:
            return gsg
        if self.reg == 1:
            return g * self.g0inv(n) * g / self.lam ** 2 + gsg
        return -1j * np.sign(nu(n, self.T)) * g * g + gsg


_MProp = MProp


def window(r: int, m: int, Nq: int) -> np.ndarray:
    """Summation indices n'' of channel r's bubble at bosonic index m: |2n'' + 1 + s m| <= 2Nq - 1,
    s = +1 for a and t (Pi symmetric about nu'' = -Omega/2), -1 for p (about +Omega/2)."""
    s = -1 if r == 1 else 1
    lo = int(np.ceil((-(2 * Nq - 1) - 1 - s * m) / 2.0))
    hi = int(np.floor(((2 * Nq - 1) - 1 - s * m) / 2.0))
    return np.arange(lo, hi + 1)


def pi_r(r: int, P: MProp, m: int, k: np.ndarray, kind: int = 0) -> np.ndarray:
    """T Pi_r(m, n'') for the window k; kind 1: the differentiated bubble S G + G S."""
    k1, k2 = (k, m - k - 1) if r == 1 else (k + m, k)
    if kind == 1:
        return P.T * (P.line(k1, 1) * P(k2) + P(k1) * P.line(k2, 1))
    return P.T * P(k1) * P(k2)


def _spin_sum(r: int, LX, LY, pi, RX, RY):
    """Literal spin sums of the three bubbles (with the channel prefactors)."""
    def mm(A, B):
        return (A * pi[None, :]) @ B
    if r == 0:
        return mm(LX, RX), mm(LX + LY, RY) + mm(LY, RX + RY)
    if r == 1:
        return 0.5 * (mm(LX, RX) + mm(LY, RY)), 0.5 * (mm(LX, RY) + mm(LY, RX))
    return -(mm(LX, RX + RY) + mm(LX + LY, RX)), -mm(LY, RY)


def bare_bubble_sum(r: int, m: int, Delta: float, T: float) -> float:
    """T sum over every n'' of the bare Pi_r(m, n''), G_0 = 1/(i nu + i Delta sgn nu) (Sec. asymptotic
    corrections: the bare bubble is known in closed form).  a and t: the n'' where both
    frequencies share a sign give digamma differences, the |m| mixed terms are summed; p: minus
    the a sum (G_0 is odd in nu)."""
    import scipy.special as sps
    ma = abs(m)
    d = Delta / (2.0 * np.pi * T)
    c = 1.0 / (2.0 * np.pi * T) ** 2
    same = c * (sps.polygamma(1, 0.5 + d) if ma == 0 else (sps.digamma(0.5 + ma + d) - sps.digamma(0.5 + d)) / ma)
    mixed = sum(1.0 / ((nu(n + ma, T) + Delta) * (nu(n, T) - Delta)) for n in range(-ma, 0))
    sa = -T * (2.0 * same + mixed)
    return -sa if r == 1 else sa


def bubble(r: int, L: MVertex, R: MVertex, P: MProp, Nq: int, kind: int = 0, tails: bool = False,
           ms=None) -> MChannel:
    """B_r(L, R) as the four asymptotic classes of channel r (kind 1: with Pi_dot).  With tails
    (kind 0 only; Sec. asymptotic corrections, the analytic-tails option) the summands beyond the
    window are added with the bare bubble: there Sigma has decayed and the vertices reach their
    values at large n'', L -> Gamma_0 + K1 + K2(m, n), R -> Gamma_0 + K1 + K2'(m, n') of the own
    channel, so each class gains its part of L(inf) t(m) R(inf) with t(m) = bare_bubble_sum - the
    window's bare sum.  ms: only these bosonic indices (the others stay zero), for samples of
    large boxes."""
    if tails and (kind != 0 or P.reg != 0):
        raise ValueError("the analytic tails are those of the bubble G G of the unregulated G_0")
    g = L.grid
    sh = g.shapes()
    out = {k: np.zeros(s, dtype=np.complex128) for k, s in sh.items()}
    nbox = np.arange(-g.N, g.N)
    own_L, own_R = L.ch[r], R.ch[r]
    for im, m in enumerate(range(-g.M, g.M + 1)):
        if ms is not None and m not in ms:
            continue
        k = window(r, m, Nq)
        pi = pi_r(r, P, m, k, kind)
        # left: rows n (the box), columns n''; L^inf(m, n'') = Gamma_0 + K1 + K2' of the own channel
        full_L = vertex_eval(L, r, m, nbox[:, None], k[None, :])
        inf_L = channel_value(own_L, g, m, 0, k, ("K1", "K2p"))
        inf_L[0] += -L.U
        inf_L[1] += L.U
        main_L = full_L - inf_L[:, None, :]
        # right: rows n'', columns n'; R^inf(m, n'') = Gamma_0 + K1 + K2 of the own channel
        full_R = vertex_eval(R, r, m, k[:, None], nbox[None, :])
        inf_R = channel_value(own_R, g, m, k, 0, ("K1", "K2"))
        inf_R[0] += -R.U
        inf_R[1] += R.U
        main_R = full_R - inf_R[:, :, None]
        x3, y3 = _spin_sum(r, main_L[0], main_L[1], pi, main_R[0], main_R[1])
        x2, y2 = _spin_sum(r, main_L[0], main_L[1], pi, inf_R[0][:, None], inf_R[1][:, None])
        x2p, y2p = _spin_sum(r, inf_L[0][None, :], inf_L[1][None, :], pi, main_R[0], main_R[1])
        x1, y1 = _spin_sum(r, inf_L[0][None, :], inf_L[1][None, :], pi, inf_R[0][:, None], inf_R[1][:, None])
        out["K3"][0, im], out["K3"][1, im] = x3, y3
        out["K2"][0, im], out["K2"][1, im] = x2[:, 0], y2[:, 0]
        out["K2p"][0, im], out["K2p"][1, im] = x2p[0], y2p[0]
        out["K1"][0, im], out["K1"][1, im] = x1[0, 0], y1[0, 0]
        if tails:
            t = np.array([bare_bubble_sum(r, m, P.Delta, P.T) - pi_r(r, MProp(P.Delta, P.T), m, k).sum()])
            lmain = channel_value(own_L, g, m, nbox, 0, ("K2",))      # [2, n]
            linf = channel_value(own_L, g, m, 0, 0, ("K1",)) + np.array([-L.U, L.U])
            rmain = channel_value(own_R, g, m, 0, nbox, ("K2p",))     # [2, n']
            rinf = channel_value(own_R, g, m, 0, 0, ("K1",)) + np.array([-R.U, R.U])
            x3, y3 = _spin_sum(r, lmain[0][:, None], lmain[1][:, None], t, rmain[0][None, :], rmain[1][None, :])
            x2, y2 = _spin_sum(r, lmain[0][:, None], lmain[1][:, None], t, np.array([[rinf[0]]]), np.array([[rinf[1]]]))
            x2p, y2p = _spin_sum(r, np.array([[linf[0]]]), np.array([[linf[1]]]), t, rmain[0][None, :], rmain[1][None, :])
            x1, y1 = _spin_sum(r, np.array([[linf[0]]]), np.array([[linf[1]]]), t, np.array([[rinf[0]]]),
                               np.array([[rinf[1]]]))
            out["K3"][0, im] += x3
            out["K3"][1, im] += y3
            out["K2"][0, im] += x2[:, 0]
            out["K2"][1, im] += y2[:, 0]
            out["K2p"][0, im] += x2p[0]
            out["K2p"][1, im] += y2p[0]
            out["K1"][0, im] += x1[0, 0]
            out["K1"][1, im] += y1[0, 0]
    return MChannel(1.0, out["K1"], out["K2"], out["K2p"], out["K3"])


def loop(V: MVertex, P: MProp, Nl: int, kind: int = 0) -> np.ndarray:
    """L(Gamma, X)(n) for n in [-N, N): T sum_{n'} [2X + Y](n, n' | n, n') X(n') over
    |2n' + 1| <= 2 Nl - 1, X = G, S or G Sigma_dot G (kind 0, 1, 2)."""
    g = V.grid
    n = np.arange(-g.N, g.N)
    k = np.arange(-Nl, Nl)
    XY = vertex_eval(V, 0, *params_of(0, n[:, None], k[None, :], n[:, None], k[None, :]))
    return P.T * ((2.0 * XY[0] + XY[1]) * P.line(k, kind)[None, :]).sum(axis=1)


def bare(grid: MGrid, U: float) -> MVertex:
    return MVertex(grid, U)


def combine(grid: MGrid, U: float, parts) -> MVertex:
    chans = [MChannel(0.0), MChannel(0.0), MChannel(0.0)]
    for r, c, coef in parts:
        chans[r] = MChannel(coef, c.K1, c.K2, c.K2p, c.K3)
    return MVertex(grid, U, chans)


def sde(V: MVertex, P: MProp, Nq: int, Nl: int) -> np.ndarray:
    """Sigma(n) = -1/2 L(B_a(Gamma_0, Gamma), G) (the a-channel form of Eq. SDE; Hartree part
    absorbed at particle-hole symmetry)."""
    phi = bubble(0, bare(V.grid, V.U), V, P, Nq)
    pv = MVertex(V.grid, 0.0, [MChannel(1.0, phi.K1, None, phi.K2p, None), MChannel(0.0), MChannel(0.0)])
    return -0.5 * loop(pv, P, Nl)


# ------------------------------------------------------------------ parquet solver
def state_pack(grid: MGrid, chans, sigma) -> np.ndarray:
    """Channels a, p, t with classes K1, K2, K2', K3 each, then Sigma [2N], one flat vector."""
    return np.concatenate([np.asarray(getattr(chans[r], c)).ravel() for r in range(3) for c in CLASSES]
                          + [np.asarray(sigma).ravel()])


def state_unpack(grid: MGrid, vec: np.ndarray):
    sh = grid.shapes()
    chans, off = [], 0
    for r in range(3):
        arrs = []
        for c in CLASSES:
            sz = int(np.prod(sh[c]))
            arrs.append(vec[off:off + sz].reshape(sh[c]))
            off += sz
        chans.append(MChannel(1.0, *arrs))
    return chans, vec[off:]


def parquet_iteration(V: MVertex, P: MProp, Nq: int, Nl: int):
    """Right-hand sides of the parquet equations in the Matsubara formalism: the symmetrized
    Bethe-Salpeter equations gamma_r' = 1/2 [B_r(I_r, Gamma) + B_r(Gamma, I_r)], I_r = Gamma
    without channel r, and the a-channel form of the SDE for Sigma (P carries Sigma)."""
    out = []
    for r in range(3):
        ir = MVertex(V.grid, V.U, [V.ch[rr] if rr != r else MChannel(0.0) for rr in range(3)])
        a = bubble(r, ir, V, P, Nq)
        b = bubble(r, V, ir, P, Nq)
        out.append(MChannel(1.0, *[0.5 * (getattr(a, c) + getattr(b, c)) for c in CLASSES]))
    return out, sde(V, P, Nq, Nl)


def pt2_state(grid: MGrid, U: float, Delta: float, Nq: int, Nl: int, reg: int = 0, lam: float = 1.0):
    """PT2 start: K1_r = B_r(Gamma_0, Gamma_0) (the other classes vanish), Sigma^(2) = SDE(Gamma_0)
    (reg 1: with G_0 -> lam G_0)."""
    g0 = bare(grid, U)
    P = MProp(Delta, grid.T, reg=reg, lam=lam)
    chans = []
    for r in range(3):
        b = bubble(r, g0, g0, P, Nq)
        chans.append(MChannel(1.0, b.K1, np.zeros_like(b.K2), np.zeros_like(b.K2p), np.zeros_like(b.K3)))
    return chans, sde(g0, P, Nq, Nl)


def parquet_solve(grid: MGrid, U: float, Delta: float, Nq: int, Nl: int, alpha: float = 0.5,
                  iterations: int = 10, tol: float = 0.0, depth: int = 0, reduce_alpha: bool = False,
                  alpha_min: float = 0.01):
    """The parquet solver of the Keldysh oracle (PT2 start, mixing or Anderson acceleration,
    residual = max over the arrays of max|F(x) - x| / max|F(x)|) on the Matsubara state, with G
    dressed by the state's Sigma on [-N, N).  Returns (channels, Sigma, residuals)."""
    from .oracle import fixed_point_solve
    chans, sigma = pt2_state(grid, U, Delta, Nq, Nl)

    def Fmap(vec):
        ch, sg = state_unpack(grid, vec)
        new, snew = parquet_iteration(MVertex(grid, U, ch), MProp(Delta, grid.T, np.array(sg)), Nq, Nl)
        return state_pack(grid, new, snew)

    def resid(x, g):
        xc, xs = state_unpack(grid, x)
        gc, gs = state_unpack(grid, g)
        worst = 0.0
        for a, f in [(getattr(xc[r], c), getattr(gc[r], c)) for r in range(3) for c in CLASSES] + [(xs, gs)]:
            md, mf = float(np.abs(f - a).max()), float(np.abs(f).max())
            worst = max(worst, md / mf if mf > 0 else (1.0 if md > 0 else 0.0))
        return worst

    x, res, _ = fixed_point_solve(Fmap, state_pack(grid, chans, sigma), resid, alpha, depth, iterations, tol,
                                  reduce_alpha, alpha_min)
    ch, sg = state_unpack(grid, x)
    return ch, np.array(sg), res


# ------------------------------------------------------------------ mfRG flow (hybridization flow)
def mloop(V: MVertex, P: MProp, Nq: int, nloops: int, centres: Optional[list] = None) -> list:
    """Multiloop insertions (Eqs. 1l-3l) in the Matsubara formalism, as in the Keldysh oracle:
    l = 1: B_r(Gamma, Gamma; Pi_dot); l = 2: B_r(gdot_rbar^(1), Gamma) + B_r(Gamma, gdot_rbar^(1));
    l >= 3: + B_r(Gamma, B_r(gdot_rbar^(l-2), Gamma)).  Returns out[l-1][r]; centre terms are
    appended to `centres` as centres[l-3][r] when it is given."""
    g = V.grid
    out = []
    for ell in range(1, nloops + 1):
        this = []
        for r in range(3):
            if ell == 1:
                this.append(bubble(r, V, V, P, Nq, 1))
                continue
            prev = out[ell - 2]
            rbar = combine(g, 0.0, [(rr, prev[rr], 1.0) for rr in range(3) if rr != r])
            Lt = bubble(r, rbar, V, P, Nq)
            Rt = bubble(r, V, rbar, P, Nq)
            tot = {k: getattr(Lt, k) + getattr(Rt, k) for k in CLASSES}
            if ell >= 3:
                rbar2 = combine(g, 0.0, [(rr, out[ell - 3][rr], 1.0) for rr in range(3) if rr != r])
                inner = bubble(r, rbar2, V, P, Nq)
                Ct = bubble(r, V, combine(g, 0.0, [(r, inner, 1.0)]), P, Nq)
                tot = {k: tot[k] + getattr(Ct, k) for k in tot}
                if centres is not None:
                    if r == 0:
                        centres.append([])
                    centres[-1].append(Ct)
            this.append(MChannel(1.0, *[tot[k] for k in CLASSES]))
        out.append(this)
    return out


def mfrg_rhs(grid: MGrid, U: float, lam: float, nloops: int, Nq: int, Nl: int, chans, sigma,
             katanin: bool = True, se_iterations: int = 0, se_atol: float = 1e-9, se_rtol: float = 1e-5,
             reg: int = 0, Delta: float = 1.0):
    """Right-hand side of the Matsubara flow in the hybridization Delta = lam (the Keldysh
    oracle's mfrg_rhs with the Matsubara bubble and loop): Sigma_dot^(1) = -L(Gamma, S),
    Gamma_dot = sum_l gdot^(l) with the l = 1 bubble along S (+ G Sigma_dot G with katanin), and
    with se_iterations (nloops >= 3) the corrections Sigma_dot_tbar = -L(gdot_{a,C} + gdot_{p,C},
    G), Sigma_dot_t = -L(Gamma, G Sigma_dot_tbar G) iterated.  reg 1: the interaction flow in lam at fixed Delta.  Returns (Gamma_dot,
    Sigma_dot)."""

    def MProp(lam_, T_, sig_, dsig_=None):  # the propagator along the flow
        return _MProp(Delta, T_, sig_, dsig_, 1, lam_) if reg == 1 else _MProp(lam_, T_, sig_, dsig_)

    V = MVertex(grid, U, chans)
    P = MProp(lam, grid.T, np.asarray(sigma))
    sd1 = -loop(V, P, Nl, 1)
    sd = sd1
    it = 0
    while True:
        Pk = MProp(lam, grid.T, np.asarray(sigma), sd if katanin else None)
        cen = []
        ins = mloop(V, Pk, Nq, nloops, centres=cen)
        if se_iterations <= 0 or nloops < 3:
            break
        ca = MChannel(1.0, *[sum(getattr(cen[l][0], c) for l in range(len(cen))) for c in CLASSES])
        cp = MChannel(1.0, *[sum(getattr(cen[l][1], c) for l in range(len(cen))) for c in CLASSES])
        tbar = -loop(MVertex(grid, 0.0, [ca, cp, MChannel(0.0)]), P, Nl, 0)
        st = -loop(V, MProp(lam, grid.T, np.asarray(sigma), tbar), Nl, 2)
        new = sd1 + tbar + st
        change = float(np.abs(new - sd).max())
        it += 1
        sd = new
        if change <= se_atol + se_rtol * float(np.abs(new).max()) or it >= se_iterations:
            break
    gdot = [MChannel(1.0, *[sum(getattr(ins[l][r], c) for l in range(nloops)) for c in CLASSES]) for r in range(3)]
    return gdot, sd


def mfrg_flow(grid: MGrid, U: float, lam_i: float, lam_f: float, steps: int, nloops: int, Nq: int, Nl: int,
              chans, sigma, katanin: bool = True, se_iterations: int = 0, adaptive: bool = False,
              atol: float = 1e-8, rtol: float = 1e-5, max_steps: int = 200, info: Optional[dict] = None,
              reg: int = 0, Delta: float = 1.0):
    """The ODE in t with Delta = Lambda(t) = 5 t|t| / sqrt(1 - t^2) (the Keldysh Delta-flow's
    parametrisation) from lam_i to lam_f: classical RK4 in `steps` equal steps, or (adaptive) the
    Cash-Karp step control of the Keldysh flow (Sec. ODE solver) with first trial step
    (t_f - t_i) / steps.  Returns (chans, sigma); info (if given) receives the accepted Delta
    values and the number of rejected steps.  reg 1: the interaction flow (G_0 -> lam G_0 at fixed
    Delta, the ODE in lam itself) from lam_i to lam_f."""
    from .oracle import flow_dlambda_dt, flow_lambda, flow_t, ode_solve

    def f(t, vec):
        ch, sg = state_unpack(grid, vec)
        gd, sd = mfrg_rhs(grid, U, flow_lambda(reg, t), nloops, Nq, Nl, ch, np.array(sg), katanin,
                          se_iterations, reg=reg, Delta=Delta)
        return flow_dlambda_dt(reg, t) * state_pack(grid, gd, sd)

    y, ts, rejected = ode_solve(f, state_pack(grid, chans, sigma), flow_t(reg, lam_i), flow_t(reg, lam_f), steps,
                                adaptive, atol, rtol, max_steps)
    if info is not None:
        info["lambdas"] = [flow_lambda(reg, t) for t in ts]
        info["rejected"] = rejected
    ch, sg = state_unpack(grid, y)
    return ch, np.array(sg)


# ------------------------------------------------------------------ susceptibilities
def chi(r: int, V: MVertex, P: MProp, Nq: int, ms=None) -> np.ndarray:
    """Susceptibility of channel r in the Matsubara formalism (Sec. Susceptibilities: the bubble
    plus bubble, vertex, bubble): chi_r^c(m) = T sum_k Pi_r(m, k) + T^2 sum_{k,l} Pi_r(m, k)
    Gamma_r^c(m; k, l) Pi_r(m, l) over the bubble's window, for the channel's two spin
    combinations c (a: X, X + 2Y; p: X + Y, X - Y; t: Y, 2X + Y).  [2, 2M + 1]; ms: only these
    bosonic indices (the others stay zero)."""
    g = V.grid
    combos = {0: ((1, 0), (1, 2)), 1: ((1, 1), (1, -1)), 2: ((0, 1), (2, 1))}[r]
    out = np.zeros((2, 2 * g.M + 1), dtype=np.complex128)
    for im, m in enumerate(range(-g.M, g.M + 1)):
        if ms is not None and m not in ms:
            continue
        k = window(r, m, Nq)
        pi = pi_r(r, P, m, k)
        XY = vertex_eval(V, r, m, k[:, None], k[None, :])
        for c, (cx, cy) in enumerate(combos):
            gam = cx * XY[0] + cy * XY[1]
            out[c, im] = pi.sum() + pi @ gam @ pi
    return out
