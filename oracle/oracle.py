"""ctypes binding of the FP64 CPU oracle (kqft_oracle.cpp) plus compositions.

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Everything here follows
the paper's definitions directly: the bubble B_r(Gamma_L, Gamma_R) (Eq. B_a and
the BSEs), the loop L(Gamma, G) (Sec. "The loop function"), the Schwinger-Dyson
equation (Eq. SDE), the susceptibility (Sec. "Susceptibilities") and the
multiloop flow equations (Eqs. 1l, 2l, 3l of the mfRG section).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kqft_oracle.cpp")
_LIB = os.path.join(_HERE, "libkqft_oracle.so")

CH = {"a": 0, "p": 1, "t": 2}
PREF = {0: 1.0, 1: 0.5, 2: -1.0}
# class bits of bubble outputs
C_K1, C_K2, C_K2P, C_K3 = 1, 2, 4, 8
C_ALL = 15
# parts of a vertex evaluation
P_R, P_K1, P_K2, P_K2P, P_K3, P_OTHER, P_ALL = 1, 2, 4, 8, 16, 32, 63


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain IEEE FP64: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OCh(C.Structure):
    _fields_ = [("coef", C.c_double), ("K1", C.c_void_p), ("K2", C.c_void_p),
                ("K2p", C.c_void_p), ("K3", C.c_void_p)]


class OVert(C.Structure):
    _fields_ = [("r0", C.c_double), ("dr0", C.c_double), ("n", C.c_int), ("L", C.c_double),
                ("a", C.c_double), ("ch", OCh * 3), ("map", C.c_int)]


class OProp(C.Structure):
    _fields_ = [("Delta", C.c_double), ("dDelta", C.c_double), ("T", C.c_double), ("eps", C.c_double),
                ("sn", C.c_int), ("sL", C.c_double), ("sa", C.c_double),
                ("SigR", C.c_void_p), ("SigK", C.c_void_p), ("reg", C.c_int), ("lam", C.c_double),
                ("dSigR", C.c_void_p), ("dSigK", C.c_void_p), ("deps", C.c_double), ("smap", C.c_int)]


class OQuad(C.Structure):
    _fields_ = [("n", C.c_int), ("map", C.c_int), ("L", C.c_double), ("a", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER
        _lib.oracle_grid_nodes.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_void_p]
        _lib.oracle_gauss_legendre.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
        _lib.oracle_quad.argtypes = [P(OQuad), C.c_void_p, C.c_void_p]
        _lib.oracle_grid_locate.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                            P(C.c_int), P(C.c_double)]
        _lib.oracle_propagator.argtypes = [C.c_int, P(OProp), C.c_int, C.c_int, C.c_void_p, C.c_void_p]
        _lib.oracle_bubble_pi.argtypes = [C.c_int, P(OProp), C.c_int, C.c_int, C.c_double, C.c_double,
                                          C.c_void_p]
        _lib.oracle_vertex_eval.argtypes = [C.c_int, P(OVert), C.c_int, C.c_uint, C.c_int, C.c_void_p,
                                            C.c_void_p]
        _lib.oracle_vertex_legs.argtypes = [P(OVert), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.oracle_bubble.argtypes = [C.c_int, C.c_int, P(OVert), P(OVert), P(OProp), C.c_int, P(OQuad),
                                       C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.oracle_bubble_points.argtypes = [C.c_int, C.c_int, P(OVert), P(OVert), P(OProp), C.c_int,
                                              P(OQuad), C.c_int, C.c_void_p, C.c_void_p]
        _lib.oracle_bubble_integrand.argtypes = [C.c_int, P(OVert), P(OVert), P(OProp), C.c_int, C.c_int,
                                                 C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        _lib.oracle_bubble_brute.argtypes = [C.c_int, P(OVert), P(OVert), P(OProp), C.c_int, P(OQuad),
                                             C.c_double, C.c_double, C.c_double, C.c_void_p]
        _lib.oracle_loop.argtypes = [C.c_int, P(OVert), P(OProp), C.c_int, P(OQuad), C.c_void_p]
        _lib.oracle_chi.argtypes = [C.c_int, P(OVert), P(OProp), P(OQuad), C.c_void_p]
        _lib.oracle_chi_points.argtypes = [P(OVert), P(OProp), P(OQuad), C.c_int, C.c_void_p, C.c_void_p]
        _lib.oracle_chi_channel.argtypes = [C.c_int, P(OVert), P(OProp), P(OQuad), C.c_int, C.c_void_p,
                                            C.c_void_p]
    return _lib


# ------------------------------------------------------------------ data model
@dataclass
class Grid:
    """Frequency grid (Sec. "Frequency grids"): x_i equidistant in [-1, 1], W_i = x_i theta with
    theta the auxiliary value of L.  map 0: v = a tan(W); map 1 (the paper's non-linear map):
    v = a W |W| / sqrt(1 - W^2)."""
    n: int
    L: float = 20.0
    a: float = 1.0
    map: int = 0

    def nodes(self) -> np.ndarray:
        out = np.zeros(self.n)
        lib().oracle_grid_nodes(self.n, self.L, self.a, self.map, out.ctypes.data)
        return out


@dataclass
class Quad:
    """n Gauss-Legendre nodes mapped by the tangent map to [-L, L] (map 0) or to R (map 1); map 2:
    the n nodes of the tangent grid Grid(n, L, a) with trapezoid weights on its auxiliary
    variable (its nodes are grid points, so vertices on that grid enter without interpolation)."""
    n: int
    map: int = 0
    L: float = 20.0
    a: float = 1.0

    def c(self) -> OQuad:
        return OQuad(self.n, self.map, self.L, self.a)

    def nodes_weights(self):
        key = (self.n, self.map, self.L, self.a)
        if key not in _QUAD_CACHE:
            v = np.zeros(self.n)
            w = np.zeros(self.n)
            lib().oracle_quad(C.byref(self.c()), v.ctypes.data, w.ctypes.data)
            _QUAD_CACHE[key] = (v, w)
        v, w = _QUAD_CACHE[key]
        return v.copy(), w.copy()


_QUAD_CACHE = {}


REG_DELTA, REG_U, REG_T, REG_NU = 0, 1, 2, 3


@dataclass
class Prop:
    """Propagator parameters (Sec. Propagator class, Sec. Flow schemes): G^R = 1/(G_0^{-1,R} -
    Sigma^R) with G_0^{-1,R} = v - eps + i Delta (regulator reg = REG_DELTA or REG_T),
    (v - eps + i Delta) / lam (REG_U) or (v - eps + i Delta)(v + i lam)/v (REG_NU); G^K by the
    general Keldysh relation with the FDR for the bath; optional dynamic Sigma on a grid and
    optional Sigma_dot there (Katanin substitution in the single-scale propagator); deps is a
    frequency-independent real part of Sigma_dot^R (the flow of the level), added to it."""
    Delta: float = 1.0
    T: float = 0.1
    eps: float = 0.0
    dDelta: float = 0.0
    sigma_grid: Optional[Grid] = None
    SigR: Optional[np.ndarray] = None
    SigK: Optional[np.ndarray] = None
    reg: int = REG_DELTA
    lam: float = 1.0
    dSigR: Optional[np.ndarray] = None
    dSigK: Optional[np.ndarray] = None
    deps: float = 0.0

    def c(self, keep: list) -> OProp:
        g = self.sigma_grid or Grid(2)
        p = OProp(self.Delta, self.dDelta, self.T, self.eps, g.n, g.L, g.a, None, None, self.reg, self.lam,
                  None, None, self.deps, g.map)
        if (self.dSigR is None) != (self.dSigK is None):
            raise ValueError("Sigma_dot needs both its retarded and its Keldysh component")
        for name in ("SigR", "SigK", "dSigR", "dSigK"):
            arr = getattr(self, name)
            if arr is not None:
                arr = _as_c(arr)
                keep.append(arr)
                setattr(p, name, arr.ctypes.data)
        return p


def _as_c(arr: np.ndarray) -> np.ndarray:
    """Complex128 arrays -> contiguous; dual arrays are float64 [..., 4] already."""
    if np.iscomplexobj(arr):
        return np.ascontiguousarray(arr, dtype=np.complex128)
    return np.ascontiguousarray(arr, dtype=np.float64)


@dataclass
class Channel:
    """gamma_r as asymptotic classes; arrays complex [2][n]..[16] (None = zero)."""
    coef: float = 1.0
    K1: Optional[np.ndarray] = None
    K2: Optional[np.ndarray] = None
    K2p: Optional[np.ndarray] = None
    K3: Optional[np.ndarray] = None


@dataclass
class Vertex:
    """Gamma = Gamma_0(r0) + sum_r coef_r gamma_r on one grid (parquet approximation R = Gamma_0)."""
    grid: Grid
    r0: float = 0.0
    ch: list = field(default_factory=lambda: [Channel(0.0), Channel(0.0), Channel(0.0)])
    dr0: float = 0.0

    def c(self, keep: list) -> OVert:
        v = OVert()
        v.r0, v.dr0, v.n, v.L, v.a = self.r0, self.dr0, self.grid.n, self.grid.L, self.grid.a
        v.map = self.grid.map
        for r in range(3):
            chn = self.ch[r]
            v.ch[r].coef = chn.coef
            for name in ("K1", "K2", "K2p", "K3"):
                arr = getattr(chn, name)
                if arr is not None and chn.coef != 0.0:
                    arr = _as_c(arr)
                    keep.append(arr)
                    setattr(v.ch[r], name, arr.ctypes.data)
                else:
                    setattr(v.ch[r], name, None)
        return v


def class_shapes(n: int):
    return {"K1": (2, n, 16), "K2": (2, n, n, 16), "K2p": (2, n, n, 16), "K3": (2, n, n, n, 16)}


def _alloc(shape, dual):
    if dual:
        return np.zeros(shape + (4,), dtype=np.float64)
    return np.zeros(shape, dtype=np.complex128)


# ------------------------------------------------------------------ primitives
def propagator(P: Prop, nu, kind: int = 0, dual: bool = False) -> np.ndarray:
    """Keldysh matrices [npts, 2, 2] of G (kind 0) or S = dG/dDelta (kind 1)."""
    keep = []
    nu = np.ascontiguousarray(np.atleast_1d(nu), dtype=np.float64)
    out = _alloc((len(nu), 2, 2), dual)
    pc = P.c(keep)
    lib().oracle_propagator(int(dual), C.byref(pc), kind, len(nu), nu.ctypes.data, out.ctypes.data)
    return out


def bubble_pi(P: Prop, r: int, w: float, vq: float, kind: int = 0) -> np.ndarray:
    keep = []
    out = np.zeros(16, dtype=np.complex128)
    pc = P.c(keep)
    lib().oracle_bubble_pi(0, C.byref(pc), r, kind, w, vq, out.ctypes.data)
    return out.reshape(4, 4)


def vertex_eval(V: Vertex, r: int, pts, parts: int = P_ALL, dual: bool = False) -> np.ndarray:
    """Vertex in channel r at points (w, v, v') -> [npts, 2, 16] (X, Y)."""
    keep = []
    pts = np.ascontiguousarray(np.atleast_2d(pts), dtype=np.float64)
    out = _alloc((len(pts), 2, 16), dual)
    vc = V.c(keep)
    lib().oracle_vertex_eval(int(dual), C.byref(vc), r, parts, len(pts), pts.ctypes.data, out.ctypes.data)
    return out


def vertex_legs(V: Vertex, al, sg, nu) -> np.ndarray:
    keep = []
    al = np.ascontiguousarray(np.atleast_2d(al), dtype=np.int32)
    sg = np.ascontiguousarray(np.atleast_2d(sg), dtype=np.int32)
    nu = np.ascontiguousarray(np.atleast_2d(nu), dtype=np.float64)
    out = np.zeros(len(al), dtype=np.complex128)
    vc = V.c(keep)
    lib().oracle_vertex_legs(C.byref(vc), len(al), al.ctypes.data, sg.ctypes.data, nu.ctypes.data, out.ctypes.data)
    return out


def bubble(r: int, left: Vertex, right: Vertex, P: Prop, q: Quad, kind: int = 0, cmask: int = C_ALL,
           dual: bool = False) -> Channel:
    """B_r(left, right) as the four asymptotic classes of channel r (coef 1)."""
    n = left.grid.n
    sh = class_shapes(n)
    out = {k: _alloc(s, dual) for k, s in sh.items()}
    keep = []
    lc, rc, pc, qc = left.c(keep), right.c(keep), P.c(keep), q.c()
    rc_ = lib().oracle_bubble(int(dual), r, C.byref(lc), C.byref(rc), C.byref(pc), kind, C.byref(qc), cmask,
                              out["K1"].ctypes.data, out["K2"].ctypes.data, out["K2p"].ctypes.data,
                              out["K3"].ctypes.data)
    if rc_ != 0:
        raise ValueError("oracle_bubble: bad arguments")
    return Channel(1.0, out["K1"], out["K2"], out["K2p"], out["K3"])


def bubble_points(r: int, left: Vertex, right: Vertex, P: Prop, q: Quad, pts, kind: int = 0,
                  dual: bool = False) -> np.ndarray:
    """Selected outputs: pts rows (class bit, iw, i, j) -> [npts, 2, 16]."""
    pts = np.ascontiguousarray(np.atleast_2d(pts), dtype=np.int32)
    out = _alloc((len(pts), 2, 16), dual)
    keep = []
    lc, rc, pc, qc = left.c(keep), right.c(keep), P.c(keep), q.c()
    lib().oracle_bubble_points(int(dual), r, C.byref(lc), C.byref(rc), C.byref(pc), kind, C.byref(qc), len(pts),
                               pts.ctypes.data, out.ctypes.data)
    return out


def bubble_integrand(r: int, left: Vertex, right: Vertex, P: Prop, pts, vq, kind: int = 0) -> np.ndarray:
    """Summand of the bubble at outputs pts[p] = (class, iw, i, j) and loop frequencies vq:
    [p][k][2 (X, Y)][16], Pi / (2 pi i) without quadrature weight."""
    pts = np.ascontiguousarray(pts, dtype=np.int32).reshape(-1, 4)
    vq = np.ascontiguousarray(np.atleast_1d(vq), dtype=np.float64)
    out = np.zeros((len(pts), len(vq), 2, 16), dtype=np.complex128)
    keep = []
    lc, rc, pc = left.c(keep), right.c(keep), P.c(keep)
    lib().oracle_bubble_integrand(r, C.byref(lc), C.byref(rc), C.byref(pc), kind, len(pts), pts.ctypes.data,
                                  len(vq), vq.ctypes.data, out.ctypes.data)
    return out


# ------------------------------------------------------------------ adaptive integration
# Gauss-Lobatto 4-point rule with its 7-point Kronrod extension and the 13-point extension of
# that (Sec. Frequency integration), on [-1, 1].  Every rule is derived from its definition:
# symmetric nodes containing the lower rule's nodes, weights and the new nodes fixed by exact
# integration of the even monomials up to the rule's degree (GL4: 5, GLK7: 9, GLK13: 18).
def _symmetric_rule(fixed, new_guess, degree):
    """Nodes = +-fixed (0 allowed), +-new; solve the even-moment equations for the new positive
    nodes and all weights (Newton from new_guess).  Returns (nodes ascending, weights)."""
    fixed = list(fixed)
    new = np.array(new_guess, dtype=float)

    def assemble(newn):
        pos = sorted(set(fixed) | set(newn.tolist()))
        return pos

    for _ in range(100):
        pos = assemble(new)
        # weights of the positive nodes (node 0 counted once) from the first len(pos) even moments
        ks = np.arange(0, degree + 1, 2)
        A = np.array([[(2.0 if x > 0 else 1.0) * x ** k for x in pos] for k in ks])
        b = np.array([2.0 / (k + 1) for k in ks])
        m = len(pos)
        if len(new) == 0:
            w = np.linalg.solve(A[:m], b[:m])
            break
        # residual of the moments as a function of the new nodes, weights eliminated from the first m moments

        def resid(newn):
            p = assemble(newn)
            Am = np.array([[(2.0 if x > 0 else 1.0) * x ** k for x in p] for k in ks])
            ww = np.linalg.solve(Am[:m], b[:m])
            return Am[m:] @ ww - b[m:], ww

        r0, w = resid(new)
        if np.abs(r0).max() < 1e-15:
            break
        J = np.zeros((len(r0), len(new)))
        h = 1e-7
        for c in range(len(new)):
            d = np.zeros_like(new)
            d[c] = h
            J[:, c] = (resid(new + d)[0] - resid(new - d)[0]) / (2 * h)
        new = new - np.linalg.lstsq(J, r0, rcond=None)[0]
    pos = assemble(new)
    nodes = np.array([-x for x in reversed(pos) if x > 0] + pos)
    wpos = dict(zip(pos, w))
    weights = np.array([wpos[abs(x)] if abs(x) in wpos else wpos[-x] for x in nodes])
    return nodes, weights


def glk_rules():
    """(GL4, GLK7, GLK13) as (nodes, weights) on [-1, 1]; GL4 and GLK7 share GLK7's nodes
    (GL4 weight 0 on the Kronrod nodes)."""
    if "rules" not in _RULES:
        gl4 = _symmetric_rule([1.0], [0.45], 5)
        glk7 = _symmetric_rule([1.0, gl4[0][-2], 0.0], [0.8], 9)
        glk13 = _symmetric_rule(list(glk7[0][glk7[0] >= 0]), [0.94, 0.64, 0.24], 18)
        w4 = np.array([dict(zip(np.round(gl4[0], 14), gl4[1])).get(round(x, 14), 0.0) for x in glk7[0]])
        _RULES["rules"] = ((glk7[0], w4), glk7, glk13)
    return _RULES["rules"]


_RULES = {}


def adaptive_glk(f, a: float, b: float, eps: float, min_width: float = 1e-12, max_depth: int = 40):
    """Adaptive Gauss-Lobatto-Kronrod integration of a vector-valued f over [a, b] (Sec. Frequency
    integration): I_s = GLK13 over [a, b] once (when it vanishes, (b - a) max|f| at its nodes
    stands in, else 1); on each interval I1 = GL4, I2 = GLK7 (same seven nodes); accept I2
    when max|I2 - I1| <= eps max|I_s|, else split at the seven nodes into six
    intervals and recurse (an interval narrower than min_width or deeper than max_depth is
    accepted as is).  f maps an array of points to [len(points), ...].
    Returns (integral, number of accepted intervals)."""
    (x7, w4), (_, w7), (x13, w13) = glk_rules()
    m, h = 0.5 * (a + b), 0.5 * (b - a)
    F13 = f(m + h * x13)
    Is = h * np.tensordot(w13, F13, axes=1)
    scale = float(np.abs(Is).max())
    if scale == 0.0:  # a vanishing estimate: the integrand's size on the domain, else 1
        scale = (b - a) * float(np.abs(F13).max()) or 1.0
    count = [0]

    def rec(lo, hi, depth):
        mm, hh = 0.5 * (lo + hi), 0.5 * (hi - lo)
        x = mm + hh * x7
        F = f(x)
        I1 = hh * np.tensordot(w4, F, axes=1)
        I2 = hh * np.tensordot(w7, F, axes=1)
        if float(np.abs(I2 - I1).max()) <= eps * scale or hi - lo < min_width or depth >= max_depth:
            count[0] += 1
            return I2
        return sum(rec(x[k], x[k + 1], depth + 1) for k in range(6))

    return rec(a, b, 0), count[0]


def bubble_adaptive_points(r: int, left: Vertex, right: Vertex, P: Prop, q: Quad, pts, eps: float, kind: int = 0):
    """Bubble outputs at pts[p] = (class, iw, i, j) by adaptive_glk over the auxiliary variable y
    of the quadrature's tangent map onto [-L, L] (v'' = a tan(y atan(L/a)), dv''/dy the
    Jacobian), each output integrated on its own: [p][2][16], and the accepted intervals."""
    if q.map != 0:
        raise ValueError("the adaptive bubble integrates over the finite tangent map")
    th = np.arctan(q.L / q.a)
    out = np.zeros((len(pts), 2, 16), dtype=np.complex128)
    counts = []
    for p, pt in enumerate(pts):
        def f(y):
            v = q.a * np.tan(y * th)
            jac = q.a * th / np.cos(y * th) ** 2
            return bubble_integrand(r, left, right, P, [pt], v, kind)[0] * jac[:, None, None]
        out[p], c = adaptive_glk(f, -1.0, 1.0, eps)
        counts.append(c)
    return out, counts


def bubble_brute(r: int, left: Vertex, right: Vertex, P: Prop, q: Quad, w: float, v: float, vp: float,
                 kind: int = 0) -> np.ndarray:
    out = np.zeros((2, 16), dtype=np.complex128)
    keep = []
    lc, rc, pc, qc = left.c(keep), right.c(keep), P.c(keep), q.c()
    lib().oracle_bubble_brute(r, C.byref(lc), C.byref(rc), C.byref(pc), kind, C.byref(qc), w, v, vp,
                              out.ctypes.data)
    return out


def loop(V: Vertex, P: Prop, q: Quad, kind: int = 0, dual: bool = False) -> np.ndarray:
    """L(Gamma, G)(v_i) as [n, 4] = Sigma^{a1'|a1} at index 2*a1'+a1 (no overall sign)."""
    out = _alloc((V.grid.n, 4), dual)
    keep = []
    vc, pc, qc = V.c(keep), P.c(keep), q.c()
    lib().oracle_loop(int(dual), C.byref(vc), C.byref(pc), kind, C.byref(qc), out.ctypes.data)
    return out


def chi(V: Vertex, P: Prop, q: Quad, dual: bool = False) -> np.ndarray:
    """Pair-space susceptibility chi_a^c(w) [2 (X, D), n, 16]."""
    out = _alloc((2, V.grid.n, 16), dual)
    keep = []
    vc, pc, qc = V.c(keep), P.c(keep), q.c()
    lib().oracle_chi(int(dual), C.byref(vc), C.byref(pc), C.byref(qc), out.ctypes.data)
    return out


def chi_points(V: Vertex, P: Prop, q: Quad, iws) -> np.ndarray:
    """chi_a^c at the listed transfer-frequency indices: [2 (X, D), len(iws), 16]."""
    iws = np.ascontiguousarray(np.atleast_1d(iws), dtype=np.int32)
    out = np.zeros((2, len(iws), 16), dtype=np.complex128)
    keep = []
    vc, pc, qc = V.c(keep), P.c(keep), q.c()
    lib().oracle_chi_points(C.byref(vc), C.byref(pc), C.byref(qc), len(iws), iws.ctypes.data, out.ctypes.data)
    return out


def chi_channel(r: int, V: Vertex, P: Prop, q: Quad, iws=None) -> np.ndarray:
    """Pair-space susceptibility of channel r (Sec. Susceptibilities: bare bubble plus bubble,
    vertex in channel r's parametrization, bubble): chi_r^c(w) = sum_k Pi_r,k + sum_{k,l} Pi_r,k
    Gamma_r^c(w; v''_k, v''_l) Pi_r,l with Pi carrying w_k/(2 pi i), for the channel's two spin
    combinations c (a: X, X + 2Y; p: X + Y, X - Y; t: Y, 2X + Y).  [2, len(iws) or n, 16]."""
    iws = np.arange(V.grid.n) if iws is None else np.atleast_1d(iws)
    iws = np.ascontiguousarray(iws, dtype=np.int32)
    out = np.zeros((2, len(iws), 16), dtype=np.complex128)
    keep = []
    vc, pc, qc = V.c(keep), P.c(keep), q.c()
    if lib().oracle_chi_channel(r, C.byref(vc), C.byref(pc), C.byref(qc), len(iws), iws.ctypes.data,
                                out.ctypes.data) != 0:
        raise ValueError("channel must be 0, 1 or 2")
    return out


# ------------------------------------------------------------------ compositions
def bare(grid: Grid, U: float, dU: float = 0.0) -> Vertex:
    """Gamma_0 only (parquet approximation R = Gamma_0)."""
    return Vertex(grid, r0=U, dr0=dU)


def pt2_k1(grid: Grid, U: float, P: Prop, q: Quad, dual: bool = False, dU: float = 0.0) -> list:
    """Second-order vertex: K1_r = B_r(Gamma_0, Gamma_0) for r = a, p, t (Sec. PT2: vertexInSOPT
    calls the bubble once per channel with two bare vertices; only K1 is non-zero)."""
    g0 = bare(grid, U, dU)
    return [bubble(r, g0, g0, P, q, 0, C_K1, dual).K1 for r in range(3)]


def seeded_vertex(grid: Grid, U: float, P: Prop, q: Quad, noise: Optional[dict] = None, dual: bool = False,
                  dU: float = 0.0) -> Vertex:
    """PT2 vertex (K1 only) plus the given noise arrays (noise[r][cls], complex)."""
    k1 = pt2_k1(grid, U, P, q, dual, dU)
    chans = []
    for r in range(3):
        cls = {"K1": k1[r], "K2": None, "K2p": None, "K3": None}
        if noise is not None:
            for name in ("K1", "K2", "K2p", "K3"):
                nz = noise[r][name]
                if dual:
                    d = np.zeros(nz.shape + (4,))
                    d[..., 0] = nz.real
                    d[..., 2] = nz.imag
                    nz = d
                cls[name] = nz if cls[name] is None else cls[name] + nz
        chans.append(Channel(1.0, cls["K1"], cls["K2"], cls["K2p"], cls["K3"]))
    return Vertex(grid, r0=U, dr0=dU, ch=chans)


def sde(V: Vertex, P: Prop, q_bubble: Quad, q_loop: Quad, dual: bool = False) -> np.ndarray:
    """Dynamic self-energy from the SDE (Eq. SDE, a-channel form):
    Sigma = -1/2 L(Phi, G) with Phi = B_a(Gamma_0, Gamma).  The Hartree loop -L(Gamma_0, G)
    equals U(<n> - 1/2) in the Keldysh-rotated basis and vanishes at particle-hole symmetry;
    the constant U/2 Hartree shift is absorbed in G_H (Sec. Hartree-Fock)."""
    g0 = bare(V.grid, V.r0, V.dr0)
    phi = bubble(0, g0, V, P, q_bubble, 0, C_K1 | C_K2P, dual)
    phi_v = Vertex(V.grid, r0=0.0, ch=[Channel(1.0, phi.K1, None, phi.K2p, None), Channel(0.0), Channel(0.0)])
    L = loop(phi_v, P, q_loop, 0, dual)
    return -0.5 * L


def sde_p(V: Vertex, P: Prop, q_bubble: Quad, q_loop: Quad) -> np.ndarray:
    """The SDE with the two lines between Gamma_0 and Gamma read as a p bubble (they run in
    the same direction): Sigma = -L(B_p(Gamma_0, Gamma), G).  B_p carries its prefactor 1/2,
    which takes the place of the symmetry factor 1/2 of the a-channel form; the loop closes the
    legs 2' and 2 as in the a-channel form.  Phi_p = B_p(Gamma_0, Gamma) has the classes K1 and
    K2' only (Gamma_0 on the left)."""
    g0 = bare(V.grid, V.r0)
    phi = bubble(1, g0, V, P, q_bubble, 0, C_K1 | C_K2P)
    phi_v = Vertex(V.grid, r0=0.0, ch=[Channel(0.0), Channel(1.0, phi.K1, None, phi.K2p, None), Channel(0.0)])
    return -loop(phi_v, P, q_loop)


def closure_2_1p(X: Vertex, P: Prop, q: Quad) -> np.ndarray:
    """The 4-point object X closed with G between its legs 2 and 1' (external legs 2' and 1),
    summed literally over the closed legs' Keldysh indices and spins (external spins up):
    out[i][2 a2' + a1] = sum_j w_j/(2 pi i) sum_{a2, a1', s} X(1' = (a1', s, v_j),
    2' = (a2', up, v_i) | 1 = (a1, up, v_i), 2 = (a2, s, v_j)) G^{a2|a1'}(v_j)."""
    g = X.grid
    v = g.nodes()
    vq, wq = q.nodes_weights()
    Gm = propagator(P, vq)
    out = np.zeros((g.n, 4), complex)
    idx = [(j, a2p, a1, a2, a1p, s) for j in range(len(vq)) for a2p in range(2) for a1 in range(2)
           for a2 in range(2) for a1p in range(2) for s in range(2)]
    al = np.array([[a1p, a2p, a1, a2] for (j, a2p, a1, a2, a1p, s) in idx])
    sg = np.array([[s, 0, 0, s] for (j, a2p, a1, a2, a1p, s) in idx])
    jj = np.array([t[0] for t in idx])
    fac = np.array([wq[j] / (2j * np.pi) * Gm[j, a2, a1p] for (j, a2p, a1, a2, a1p, s) in idx])
    slot = np.array([2 * a2p + a1 for (j, a2p, a1, a2, a1p, s) in idx])
    for i in range(g.n):
        nu = np.stack([vq[jj], np.full(len(jj), v[i]), np.full(len(jj), v[i]), vq[jj]], axis=1)
        vals = vertex_legs(X, al, sg, nu) * fac
        out[i] = np.bincount(slot, weights=vals.real, minlength=4) + 1j * np.bincount(slot, weights=vals.imag,
                                                                                        minlength=4)
    return out


def sde_t(V: Vertex, P: Prop, q_bubble: Quad, q_loop: Quad) -> np.ndarray:
    """The SDE with the two lines between Gamma_0 and Gamma read as a t bubble: Phi_t =
    B_t(Gamma_0, Gamma), closed between its legs 2 and 1' (which puts Gamma_0's outgoing leg and
    Gamma's incoming leg outside, the topology of the SDE), Sigma = +1/2 of that closure (the
    crossed closure flips the sign of the a-channel form's -1/2)."""
    g0 = bare(V.grid, V.r0)
    phi = bubble(2, g0, V, P, q_bubble, 0, C_K1 | C_K2P)
    phi_v = Vertex(V.grid, r0=0.0, ch=[Channel(0.0), Channel(0.0), Channel(1.0, phi.K1, None, phi.K2p, None)])
    return 0.5 * closure_2_1p(phi_v, P, q_loop)


def sde_average(V: Vertex, P: Prop, q_bubble: Quad, q_loop: Quad) -> np.ndarray:
    """The three ways of evaluating the SDE (its two inner lines read as an a, a p or a t bubble)
    combined with equal weights (Sec. parquet solver).  Equal in the continuum; on a grid they
    differ by the discretisation of the bubble, and their mean cancels the part that breaks the
    evenness of Sigma in U at particle-hole symmetry at third order."""
    return (sde(V, P, q_bubble, q_loop) + sde_p(V, P, q_bubble, q_loop) + sde_t(V, P, q_bubble, q_loop)) / 3.0


def chi_scalar(chi_pair: np.ndarray) -> np.ndarray:
    """chi^R(w) = u^T chi v with u on pairs {(0,0),(1,1)} and v on {(0,1),(1,0)}."""
    m = chi_pair.reshape(chi_pair.shape[:-1] + (4, 4))
    return m[..., [0, 3], :][..., :, [1, 2]].sum(axis=(-1, -2))


def combine(grid: Grid, parts: Sequence[tuple], r0: float = 0.0) -> Vertex:
    """Vertex from (channel index, Channel, coefficient) triples."""
    chans = [Channel(0.0), Channel(0.0), Channel(0.0)]
    for r, chn, c in parts:
        chans[r] = Channel(c, chn.K1, chn.K2, chn.K2p, chn.K3)
    return Vertex(grid, r0=r0, ch=chans)


def mloop(V: Vertex, P: Prop, q: Quad, nloops: int, dual: bool = False, centres: Optional[list] = None) -> list:
    """Multiloop insertions (mfRG flow equations, Eqs. 1l-3l):
      l = 1: gdot_r = B_r(Gamma, Gamma; Pidot),
      l = 2: gdot_r = B_r(gdot_rbar^(1), Gamma) + B_r(Gamma, gdot_rbar^(1)),
      l >= 3: + B_r(Gamma, B_r(gdot_rbar^(l-2), Gamma)) (the centre term, as two explicit bubbles),
    where gdot_rbar = sum of the two other channels.  Returns out[l-1][r] (Channel).  When a
    list is given as `centres`, the centre terms are appended to it as centres[l-3][r]."""
    g = V.grid
    out = []
    for ell in range(1, nloops + 1):
        this = []
        for r in range(3):
            if ell == 1:
                this.append(bubble(r, V, V, P, q, 1, C_ALL, dual))
                continue
            prev = out[ell - 2]
            rbar = combine(g, [(rr, prev[rr], 1.0) for rr in range(3) if rr != r])
            Lt = bubble(r, rbar, V, P, q, 0, C_ALL, dual)
            Rt = bubble(r, V, rbar, P, q, 0, C_ALL, dual)
            tot = {k: getattr(Lt, k) + getattr(Rt, k) for k in ("K1", "K2", "K2p", "K3")}
            if ell >= 3:
                prev2 = out[ell - 3]
                rbar2 = combine(g, [(rr, prev2[rr], 1.0) for rr in range(3) if rr != r])
                inner = bubble(r, rbar2, V, P, q, 0, C_ALL, dual)
                Ct = bubble(r, V, combine(g, [(r, inner, 1.0)]), P, q, 0, C_ALL, dual)
                tot = {k: tot[k] + getattr(Ct, k) for k in tot}
                if centres is not None:
                    if r == 0:
                        centres.append([])
                    centres[-1].append(Ct)
            this.append(Channel(1.0, tot["K1"], tot["K2"], tot["K2p"], tot["K3"]))
        out.append(this)
    return out


def to_dual(arr: Optional[np.ndarray]) -> Optional[np.ndarray]:
    """Complex array -> dual layout [..., 4] = (re, d re, im, d im) with zero derivative."""
    if arr is None:
        return None
    d = np.zeros(arr.shape + (4,))
    d[..., 0] = arr.real
    d[..., 2] = arr.imag
    return d


def dual_parts(d: np.ndarray):
    """(value, derivative) complex arrays of a dual array."""
    return d[..., 0] + 1j * d[..., 2], d[..., 1] + 1j * d[..., 3]


def dual_vertex(V: Vertex, dr0: float = 0.0) -> Vertex:
    chans = [Channel(c.coef, *[to_dual(getattr(c, k)) for k in ("K1", "K2", "K2p", "K3")]) for c in V.ch]
    return Vertex(V.grid, V.r0, chans, dr0=dr0)


# ------------------------------------------------------------------ crossed closure
def t_closure(X: Vertex, P: Prop, q: Quad) -> np.ndarray:
    """The 4-point object X closed with G between its legs 2' and 1 (external legs 1' and 2),
    summed literally over the closed legs' Keldysh indices and spins (external spins up):
    out[i][2 a1' + a2] = sum_j w_j/(2 pi i) sum_{a1, a2', s} X(1' = (a1', up, v_i),
    2' = (a2', s, v_j) | 1 = (a1, s, v_j), 2 = (a2, up, v_i)) G^{a1|a2'}(v_j)."""
    g = X.grid
    v = g.nodes()
    vq, wq = q.nodes_weights()
    Gm = propagator(P, vq)
    out = np.zeros((g.n, 4), complex)
    idx = [(j, a1p, a2, a2p, a1, s) for j in range(len(vq)) for a1p in range(2) for a2 in range(2)
           for a2p in range(2) for a1 in range(2) for s in range(2)]
    for i in range(g.n):
        al = np.array([[a1p, a2p, a1, a2] for (j, a1p, a2, a2p, a1, s) in idx])
        sg = np.array([[0, s, s, 0] for (j, a1p, a2, a2p, a1, s) in idx])
        nu = np.array([[v[i], vq[j], vq[j], v[i]] for (j, a1p, a2, a2p, a1, s) in idx])
        vals = vertex_legs(X, al, sg, nu)
        for val, (j, a1p, a2, a2p, a1, s) in zip(vals, idx):
            out[i, 2 * a1p + a2] += wq[j] / (2j * np.pi) * val * Gm[j, a1, a2p]
    return out


# ------------------------------------------------------------------ Hartree term
def occupation(E: float, Delta: float, T: float, q: Quad, grid: Optional[Grid] = None,
               sigma: Optional[np.ndarray] = None) -> float:
    """<n_sigma> of G^R = 1/(v - E + i Delta - Sigma^R_dyn(v)) (Eq. Hartree with G^< = -2i n_F Im G^R
    in equilibrium, Sec. Hartree-Fock), written with n_F = (1 - tanh(v/2T))/2 and the spectral sum
    rule int A = 1 for the constant half: <n> = 1/2 + (1/2 pi) int dv tanh(v/2T) Im G^R(v).  The two
    forms agree for every causal G; this one keeps <n> = 1/2 exact at particle-hole symmetry when
    Sigma is only known on a grid.  Quadrature q: the full-line map (Lorentzian tails)."""
    v, w = q.nodes_weights()
    P = sigma_prop(grid, Delta, T, sigma) if sigma is not None else Prop(Delta, T)
    P.eps = E
    GR = propagator(P, v)[:, 1, 0]
    return float(0.5 + np.sum(w * np.tanh(v / (2.0 * T)) * GR.imag) / (2.0 * np.pi))


def hartree(U: float, eps_d: float, Delta: float, T: float, q: Quad, grid: Optional[Grid] = None,
            sigma: Optional[np.ndarray] = None, self_consistent: bool = True, tol: float = 1e-12,
            sigma_H: float = 0.0, max_iterations: int = 200):
    """Hartree term Sigma_H = U <n_sigma> of the level eps_d (Sec. Hartree-Fock, Eq. Hartree) with
    the dynamic self-energy sigma ([n, 4] on grid, or none).  One-shot: U n(eps_d + sigma_H).
    Self-consistent: bisection of f(x) = x - U n(eps_d + x) on [0, U] (f(0) <= 0 <= f(U) for
    U >= 0, f increasing) until the bracket is narrower than tol.  Returns (Sigma_H, steps)."""
    if U < 0:
        raise ValueError("the bracketing assumes U >= 0")
    if not self_consistent:
        return U * occupation(eps_d + sigma_H, Delta, T, q, grid, sigma), 1
    lo, hi = 0.0, U
    it = 0
    while hi - lo > tol and it < max_iterations:
        mid = 0.5 * (lo + hi)
        if mid - U * occupation(eps_d + mid, Delta, T, q, grid, sigma) > 0.0:
            hi = mid
        else:
            lo = mid
        it += 1
    return 0.5 * (lo + hi), it


# ------------------------------------------------------------------ parquet iteration
CLASSES = ("K1", "K2", "K2p", "K3")


def sigma_prop(grid: Grid, Delta: float, T: float, sigma: Optional[np.ndarray]) -> Prop:
    """Propagator with a dynamic self-energy given on the vertex grid as [n, 4] (index 2*a'+a:
    Sigma^K at 0, Sigma^R at 1), linearly interpolated on the auxiliary variable."""
    if sigma is None:
        return Prop(Delta, T)
    return Prop(Delta, T, sigma_grid=grid, SigR=np.ascontiguousarray(sigma[:, 1]),
                SigK=np.ascontiguousarray(sigma[:, 0]))


def parquet_iteration(V: Vertex, P: Prop, q_bubble: Quad, q_loop: Quad, sde_forms: int = 1):
    """Right-hand sides of the parquet equations for the state (Gamma, Sigma) (Sec. parquet
    solver): the Bethe-Salpeter equations gamma_r = I_r Pi_r Gamma with the irreducible vertex
    I_r = Gamma - gamma_r, symmetrized as 1/2 [B_r(I_r, Gamma) + B_r(Gamma, I_r)], and the
    Schwinger-Dyson equation for Sigma: its a-channel form, or with sde_forms = 3 the mean of
    its three forms.  P carries Sigma of the state.
    Returns ([gamma_a', gamma_p', gamma_t'] as Channels, Sigma' [n, 4])."""
    if sde_forms not in (1, 3):
        raise ValueError("sde_forms must be 1 or 3")
    g = V.grid
    out = []
    for r in range(3):
        ir = Vertex(g, V.r0, [V.ch[rr] if rr != r else Channel(0.0) for rr in range(3)])
        a = bubble(r, ir, V, P, q_bubble)
        b = bubble(r, V, ir, P, q_bubble)
        out.append(Channel(1.0, *[0.5 * (getattr(a, c) + getattr(b, c)) for c in CLASSES]))
    return out, (sde_average if sde_forms == 3 else sde)(V, P, q_bubble, q_loop)


class AndersonMixer:
    """One step of mixing or Anderson acceleration (Walker and Ni 2011) per call, over the real
    inner product Re <a, b> of complex vectors: from x_k and g_k = F(x_k), f_k = g_k - x_k; the
    columns dF_i = f_{i+1} - f_i, dG_i = g_{i+1} - g_i of the last `depth` calls; gamma from the
    normal equations (dF^T dF + eps I) gamma = dF^T f_k with eps = 1e-14 max_i (dF^T dF)_ii;
        x_{k+1} = x_k + alpha f_k - sum_i gamma_i (dG_i - (1 - alpha) dF_i);
    depth 0 (or an empty history) is linear mixing x_{k+1} = x_k + alpha f_k.  reset() clears
    the history (the next call still records its f, g for the following one)."""

    def __init__(self, depth: int, alpha: float):
        self.depth, self.alpha = depth, alpha
        self.dF, self.dG = [], []
        self.f_prev = self.g_prev = None

    def reset(self):
        self.dF, self.dG = [], []

    def step(self, x: np.ndarray, g: np.ndarray, record: bool = True) -> np.ndarray:
        f = g - x
        if record and self.depth > 0 and self.f_prev is not None:
            self.dF.append(f - self.f_prev)
            self.dG.append(g - self.g_prev)
            if len(self.dF) > self.depth:
                self.dF.pop(0)
                self.dG.pop(0)
        self.f_prev, self.g_prev = f, g
        step = x + self.alpha * f
        if self.dF:
            m = len(self.dF)
            A = np.array([[np.vdot(self.dF[i], self.dF[j]).real for j in range(m)] for i in range(m)])
            b = np.array([np.vdot(self.dF[i], f).real for i in range(m)])
            A = A + 1e-14 * A.diagonal().max() * np.eye(m)
            gam = np.linalg.solve(A, b)
            for i in range(m):
                step = step - gam[i] * (self.dG[i] - (1.0 - self.alpha) * self.dF[i])
        return step


def fixed_point_solve(Fmap, x0: np.ndarray, residual, alpha: float = 0.5, depth: int = 0, iterations: int = 10,
                      tol: float = 0.0, reduce_alpha: bool = False, alpha_min: float = 0.01):
    """Fixed-point iteration x = F(x) on complex vectors (Sec. parquet solver: mixing and
    Anderson acceleration).  Per iteration k: g_k = F(x_k), r_k = residual(x_k, g_k), then one
    AndersonMixer step of the given depth and mixing factor.  With reduce_alpha, r_k > r_{k-1}
    halves alpha (not below alpha_min) and clears the Anderson history before the step.  Stops
    after the update of the first iteration with r_k < tol.  Returns (x, residuals, final alpha)."""
    x = x0
    res = []
    mix = AndersonMixer(depth, alpha)
    for k in range(iterations):
        g = Fmap(x)
        r = residual(x, g)
        grew = reduce_alpha and res and r > res[-1]
        if grew:
            mix.alpha = max(0.5 * mix.alpha, alpha_min)
            mix.reset()
        res.append(r)
        x = mix.step(x, g, record=not grew)
        if r < tol:
            break
    return x, res, mix.alpha


def _rel_residual(n: int):
    """max over the arrays of max|F - x| / max|F| (three channels x four classes, Sigma)."""
    def resid(x, g):
        xc, xs = state_unpack(x, n)
        gc, gs = state_unpack(g, n)
        worst = 0.0
        pairs = [(getattr(xc[r], c), getattr(gc[r], c)) for r in range(3) for c in CLASSES] + [(xs, gs)]
        for a, f in pairs:
            md, mf = float(np.abs(f - a).max()), float(np.abs(f).max())
            worst = max(worst, md / mf if mf > 0 else (1.0 if md > 0 else 0.0))
        return worst
    return resid


def parquet_solve(grid: Grid, U: float, Delta: float, T: float, q_bubble: Quad, q_loop: Quad,
                  alpha: float = 0.5, iterations: int = 10, tol: float = 0.0, depth: int = 0,
                  reduce_alpha: bool = False, alpha_min: float = 0.01, eps_d: Optional[float] = None,
                  q_hartree: Optional[Quad] = None, hartree_tol: float = 1e-12, sde_forms: int = 1):
    """Parquet solver (Sec. parquet solver): start from PT2 (vertex K1 in every channel,
    Sigma^(2) from the SDE of Gamma_0), then fixed_point_solve on the state (three channels,
    Sigma) with F = parquet_iteration at the propagator dressed by the state's Sigma; the
    residual is the relative max-norm change, max over the arrays of ||F(x) - x|| / ||F(x)||.
    With eps_d (the asymmetric model, Sec. Hartree-Fock) the level of G is eps_d + Sigma_H:
    the PT2 start takes the self-consistent Sigma_H of the bare level, the state carries
    Sigma_H as one more entry, and F updates it once per iteration (one shot, U <n> of the
    state's propagator).  Without eps_d the level is 0 (particle-hole symmetry).  sde_forms = 3
    takes Sigma from the mean of the SDE's three forms (the PT2 start is the same: the forms agree
    at second order).
    Returns (channels, Sigma, residuals per step), plus Sigma_H with eps_d."""
    n = grid.n
    aam = eps_d is not None
    sH = 0.0
    if aam:
        sH, _ = hartree(U, eps_d, Delta, T, q_hartree, tol=hartree_tol)
    chans, sigma = pt2_state(grid, U, Delta, T, q_bubble, q_loop, eps=(eps_d + sH) if aam else 0.0)

    def Fmap(vec):
        ch, sg = state_unpack(vec[:-1] if aam else vec, n)
        P = sigma_prop(grid, Delta, T, sg)
        if aam:
            P.eps = eps_d + vec[-1].real
        new, snew = parquet_iteration(Vertex(grid, U, ch), P, q_bubble, q_loop, sde_forms)
        out = state_pack(new, snew)
        if aam:
            h, _ = hartree(U, eps_d, Delta, T, q_hartree, grid, sg, self_consistent=False, sigma_H=vec[-1].real)
            out = np.concatenate([out, [h + 0j]])
        return out

    base = _rel_residual(n)

    def resid(x, g):
        if not aam:
            return base(x, g)
        r = base(x[:-1], g[:-1])
        md, mf = abs(g[-1] - x[-1]), abs(g[-1])
        return max(r, md / mf if mf > 0 else (1.0 if md > 0 else 0.0))

    x0 = state_pack(chans, sigma)
    if aam:
        x0 = np.concatenate([x0, [sH + 0j]])
    x, res, _ = fixed_point_solve(Fmap, x0, resid, alpha, depth, iterations, tol, reduce_alpha, alpha_min)
    ch, sg = state_unpack(x[:-1] if aam else x, n)
    if aam:
        return ch, sg, res, float(x[-1].real)
    return ch, sg, res


# ------------------------------------------------------------------ mfRG flow
def pt2_state(grid: Grid, U: float, Delta: float, T: float, q_bubble: Quad, q_loop: Quad, eps: float = 0.0):
    """PT2 state (Sec. PT2): K1_r = B_r(Gamma_0, Gamma_0) in every channel, Sigma^(2) from the
    SDE of Gamma_0 with the Hartree propagator (level eps = eps_d + Sigma_H)."""
    P0 = Prop(Delta, T, eps=eps)
    k1 = pt2_k1(grid, U, P0, q_bubble)
    z2 = np.zeros((2, grid.n, grid.n, 16), complex)
    chans = [Channel(1.0, k1[r], z2.copy(), z2.copy(), np.zeros((2, grid.n, grid.n, grid.n, 16), complex))
             for r in range(3)]
    return chans, sde(bare(grid, U), P0, q_bubble, q_loop)


# Regulators of the flow (Sec. Flow schemes) and the flow parameter of the ODE solver
# (Sec. Details on the ODE solver): the Delta-flow integrates in t with
# Lambda(t) = 5 t |t| / sqrt(1 - t^2); the other flows integrate in Lambda itself.
def flow_lambda(reg: int, t: float) -> float:
    return 5.0 * t * abs(t) / np.sqrt(1.0 - t * t) if reg == REG_DELTA else t


def flow_t(reg: int, lam: float) -> float:
    """Inverse of flow_lambda: 25 t^4 + Lambda^2 t^2 - Lambda^2 = 0 for the Delta-flow."""
    if reg != REG_DELTA:
        return lam
    l2 = lam * lam
    return float(np.sign(lam) * np.sqrt((-l2 + np.sqrt(l2 * l2 + 100.0 * l2)) / 50.0))


def flow_dlambda_dt(reg: int, t: float) -> float:
    return 5.0 * abs(t) * (2.0 - t * t) / (1.0 - t * t) ** 1.5 if reg == REG_DELTA else 1.0


def flow_prop(grid: Grid, reg: int, lam: float, Delta: float, T: float, sigma, dsigma=None, eps: float = 0.0,
              deps: float = 0.0) -> Prop:
    """Propagator at flow parameter lam: the hybridization for the Delta-flow, the
    temperature for the T-flow, the regulator parameter of the interaction and frequency flows;
    level eps, and deps the flow of the level in the G Sigma_dot G line."""
    P = sigma_prop(grid, Delta, T, sigma)
    P.eps, P.deps = eps, deps
    if reg == REG_DELTA:
        P.Delta = lam
    elif reg == REG_T:
        P.T = lam
    P.reg, P.lam = reg, lam if reg in (REG_U, REG_NU) else 1.0
    if dsigma is not None:
        P.sigma_grid = grid
        P.dSigR = np.ascontiguousarray(dsigma[:, 1])
        P.dSigK = np.ascontiguousarray(dsigma[:, 0])
    return P


def state_pack(chans, sigma) -> np.ndarray:
    """Flat state vector: channels a, p, t with classes K1, K2, K2', K3 each, then Sigma."""
    return np.concatenate([getattr(chans[r], c).ravel() for r in range(3) for c in CLASSES] + [sigma.ravel()])


def state_unpack(vec: np.ndarray, n: int):
    shapes = class_shapes(n)
    chans, off = [], 0
    for r in range(3):
        arrs = []
        for c in CLASSES:
            sz = int(np.prod(shapes[c]))
            arrs.append(vec[off:off + sz].reshape(shapes[c]))
            off += sz
        chans.append(Channel(1.0, *arrs))
    return chans, vec[off:].reshape(n, 4)


@dataclass
class FlowOptions:
    """Options of the mfRG flow: regulator, Katanin substitution, self-energy corrections
    (iterated while the max-norm change of Sigma_dot exceeds se_atol + se_rtol max|Sigma_dot|,
    at most se_iterations times; 0 = none) and the ODE method (fixed-step classical RK4 or
    Cash-Karp with step control on max_i |err_i| / (atol + rtol max(|y_i|, |y4_i|)))."""
    reg: int = REG_DELTA
    Delta: float = 1.0  # the hybridization of the flows other than the Delta-flow
    katanin: bool = True
    se_iterations: int = 0
    se_atol: float = 1e-9
    se_rtol: float = 1e-5
    se_anderson: int = 0  # Anderson depth of the self-energy correction iterations (0: plain)
    adaptive: bool = False
    atol: float = 1e-8
    rtol: float = 1e-5
    max_steps: int = 200


def loop_static(V: Vertex, P: Prop, q: Quad, kind: int = 0) -> np.ndarray:
    """The loop L(Gamma, X) for |v| beyond the grid, its asymptotic value (Sec. loop function: for
    the asymmetric model it is taken from the Hartree term and the t-channel classes).  In the
    loop's legs (v, v_j | v, v_j) the t channel has transfer frequency 0 and first fermionic
    frequency v_j, so Gamma_0, K1_t(0) and K2_t(0, v_j) do not depend on v; every other class is
    read at a frequency that grows with v and is zero beyond the grid.  Returns the [4] vector
    (index 2 a1' + a1): the loop of that static part of Gamma, the same at every grid point."""
    t = V.ch[2]
    sv = Vertex(V.grid, V.r0, [Channel(0.0), Channel(0.0), Channel(t.coef, t.K1, t.K2, None, None)], dr0=V.dr0)
    return loop(sv, P, q, kind)[0]


def _split_level(full: np.ndarray, s: float) -> np.ndarray:
    """Sigma_dot on the grid minus the real constant s in its retarded and advanced components."""
    out = full.copy()
    out[:, 1] -= s
    out[:, 2] -= s
    return out


def mfrg_rhs(grid: Grid, U: float, T: float, lam: float, nloops: int, q_bubble: Quad, q_loop: Quad, chans, sigma,
             fo: Optional[FlowOptions] = None, info: Optional[dict] = None, eps: Optional[float] = None):
    """Right-hand side of the flow (Sec. mfRG) at flow parameter lam:
      Sigma_dot^(1) = -L(Gamma, S)                            (one-loop self-energy flow)
      Gamma_dot     = sum_{l <= nloops} gdot^(l), with the l = 1 bubble differentiated along
                      S + G Sigma_dot G (Katanin) or S
    and, with self-energy corrections (nloops >= 3), iterated from there:
      Sigma_dot_tbar = -L(gdot_{a,C} + gdot_{p,C}, G)          (centre terms summed over l)
      Sigma_dot_t    = -L(Gamma, G Sigma_dot_tbar G)
      Sigma_dot      = Sigma_dot^(1) + Sigma_dot_tbar + Sigma_dot_t,
    re-evaluating Gamma_dot with the new Sigma_dot after each update.  The correction loop is
    the fixed-point iteration Sigma_dot = F(Sigma_dot); with se_anderson > 0 the next iterate
    is the AndersonMixer step (mixing factor 1) of that depth instead of F(Sigma_dot) itself,
    and the right-hand side returned is still F of the last iterate with its Gamma_dot.

    With eps (the asymmetric model, level eps = eps_d + Sigma_inf of G) the self-energy is split
    into the real constant Sigma_inf, its value beyond the grid, and the rest on the grid: every
    loop L contributes ds = -Re of the retarded component of its asymptotic value (loop_static)
    to d Sigma_inf and its grid values minus ds (retarded and advanced components) to the rest;
    the G Sigma_dot G lines carry both (ds as the flow of the level).  The correction loop
    -L(gdot_{a,C} + gdot_{p,C}, G) has no asymptotic part (no bare vertex, no t channel).
    Returns (Gamma_dot, Sigma_dot of the rest), plus d Sigma_inf when eps is given."""
    fo = fo or FlowOptions()
    aam = eps is not None
    e0 = eps if aam else 0.0
    P = flow_prop(grid, fo.reg, lam, fo.Delta, T, sigma, eps=e0)
    V = Vertex(grid, U, chans)

    def part(Px, kind):
        full = -loop(V, Px, q_loop, kind=kind)
        if not aam:
            return full, 0.0
        ds = float((-loop_static(V, Px, q_loop, kind))[1].real)
        return _split_level(full, ds), ds

    sd1, ds1 = part(P, 1)
    sd, ds = sd1, ds1
    it = 0
    mixer = AndersonMixer(fo.se_anderson, 1.0)
    while True:
        Pk = flow_prop(grid, fo.reg, lam, fo.Delta, T, sigma, sd if fo.katanin else None, eps=e0,
                       deps=ds if fo.katanin else 0.0)
        cen = []
        ins = mloop(V, Pk, q_bubble, nloops, centres=cen)
        if fo.se_iterations <= 0 or nloops < 3:
            break
        ca = Channel(1.0, *[sum(getattr(cen[l][0], c) for l in range(len(cen))) for c in CLASSES])
        cp = Channel(1.0, *[sum(getattr(cen[l][1], c) for l in range(len(cen))) for c in CLASSES])
        tbar = -loop(Vertex(grid, 0.0, [ca, cp, Channel(0.0)]), P, q_loop, kind=0)
        st, dst = part(flow_prop(grid, fo.reg, lam, fo.Delta, T, sigma, tbar, eps=e0), 2)
        new, dnew = sd1 + tbar + st, ds1 + dst
        change = max(float(np.abs(new - sd).max()), abs(dnew - ds))
        it += 1
        if change <= fo.se_atol + fo.se_rtol * max(float(np.abs(new).max()), abs(dnew)) or it >= fo.se_iterations:
            sd, ds = new, dnew
            break
        if fo.se_anderson > 0:
            if aam:
                mixed = mixer.step(np.concatenate([sd.ravel(), [ds + 0j]]), np.concatenate([new.ravel(), [dnew + 0j]]))
                sd, ds = mixed[:-1].reshape(sd.shape), float(mixed[-1].real)
            else:
                sd = mixer.step(sd, new)
        else:
            sd, ds = new, dnew
    if info is not None:
        info["se_iterations"] = info.get("se_iterations", 0) + it
        info["rhs"] = info.get("rhs", 0) + 1
    gdot = [Channel(1.0, *[sum(getattr(ins[l][r], c) for l in range(nloops)) for c in CLASSES]) for r in range(3)]
    return (gdot, sd, ds) if aam else (gdot, sd)


# Cash-Karp embedded Runge-Kutta pair (Cash and Karp 1990): nodes, stage matrix, weights of
# the fifth- and of the fourth-order solution.
CK_C = (0.0, 1 / 5, 3 / 10, 3 / 5, 1.0, 7 / 8)
CK_A = ((),
        (1 / 5,),
        (3 / 40, 9 / 40),
        (3 / 10, -9 / 10, 6 / 5),
        (-11 / 54, 5 / 2, -70 / 27, 35 / 27),
        (1631 / 55296, 175 / 512, 575 / 13824, 44275 / 110592, 253 / 4096))
CK_B5 = (37 / 378, 0.0, 250 / 621, 125 / 594, 0.0, 512 / 1771)
CK_B4 = (2825 / 27648, 0.0, 18575 / 48384, 13525 / 55296, 277 / 14336, 1 / 4)


def ode_solve(f, y0: np.ndarray, t0: float, t1: float, steps: int, adaptive: bool = False, atol: float = 1e-8,
              rtol: float = 1e-5, max_steps: int = 200):
    """Integrate y' = f(t, y) from t0 to t1.  Fixed: classical RK4 in `steps` equal steps.
    Adaptive: Cash-Karp, advancing with the fourth-order solution; err = max_i |e_i| /
    (atol + rtol max(|y_i|, |y4_i|)) (entries with e_i = 0 count as 0, a NaN makes err
    infinite) with e = h sum_j (b5_j - b4_j) k_j; accept when err <= 1
    and grow h by min(5, 0.9 err^(-1/5)), else shrink by max(0.1, 0.9 err^(-1/4)) and retry;
    the first trial step is (t1 - t0) / steps and the last one is cut to land on t1.
    Returns (y, accepted t values including t0, number of rejected steps)."""
    y, t = y0, t0
    ts = [t0]
    if not adaptive:
        h = (t1 - t0) / steps
        for st in range(steps):
            ta = t0 + st * h
            k1 = f(ta, y)
            k2 = f(ta + h / 2, y + (h / 2) * k1)
            k3 = f(ta + h / 2, y + (h / 2) * k2)
            k4 = f(ta + h, y + h * k3)
            y = y + (h / 6) * k1 + (h / 3) * k2 + (h / 3) * k3 + (h / 6) * k4
            ts.append(t0 + (st + 1) * h)
        return y, ts, 0
    h = (t1 - t0) / steps
    rejected, k1 = 0, None
    for _ in range(max_steps):
        last = (t + h - t1) * np.sign(t1 - t0) >= 0.0
        if last:
            h = t1 - t
        if k1 is None:
            k1 = f(t, y)
        ks = [k1]
        for i in range(1, 6):
            yi = y + h * sum(a * k for a, k in zip(CK_A[i], ks))
            ks.append(f(t + CK_C[i] * h, yi))
        y4 = y + h * sum(b * k for b, k in zip(CK_B4, ks))
        e = h * sum((b5 - b4) * k for b5, b4, k in zip(CK_B5, CK_B4, ks))
        ae = np.abs(e)
        with np.errstate(invalid="ignore", divide="ignore"):
            ratio = np.where(ae == 0.0, 0.0, ae / (atol + rtol * np.maximum(np.abs(y), np.abs(y4))))
        err = float(ratio.max())
        if not np.isfinite(err):
            err = np.inf
        if err <= 1.0:
            y, t, k1 = y4, (t1 if last else t + h), None
            ts.append(t)
            if last:
                return y, ts, rejected
            h *= 5.0 if err == 0.0 else min(5.0, 0.9 * err ** -0.2)
        else:
            rejected += 1
            h *= max(0.1, 0.9 * err ** -0.25)
    raise RuntimeError("ode_solve: step limit reached")


def mfrg_flow(grid: Grid, U: float, T: float, lam_i: float, lam_f: float, steps: int, nloops: int,
              q_bubble: Quad, q_loop: Quad, chans, sigma, fo: Optional[FlowOptions] = None,
              eps_d: Optional[float] = None, sigma_inf: float = 0.0):
    """Integrate the flow (mfrg_rhs) of the state (chans, sigma) from lam_i to lam_f (Sec. ODE
    solver).  With eps_d, the asymmetric model: the state carries the real constant sigma_inf
    (the self-energy beyond the grid; the level of G is eps_d + sigma_inf) as one more entry,
    and sigma is the rest on the grid.  Returns (chans, sigma, info) with info["lambdas"] the
    accepted flow parameters and, with eps_d, info["sigma_inf"]."""
    fo = fo or FlowOptions()
    n = grid.n
    info = {}
    aam = eps_d is not None

    def f(t, vec):
        if aam:
            ch, sg = state_unpack(vec[:-1], n)
            gd, sd, ds = mfrg_rhs(grid, U, T, flow_lambda(fo.reg, t), nloops, q_bubble, q_loop, ch, sg, fo, info,
                                  eps=eps_d + vec[-1].real)
            return flow_dlambda_dt(fo.reg, t) * np.concatenate([state_pack(gd, sd), [ds + 0j]])
        ch, sg = state_unpack(vec, n)
        gd, sd = mfrg_rhs(grid, U, T, flow_lambda(fo.reg, t), nloops, q_bubble, q_loop, ch, sg, fo, info)
        return flow_dlambda_dt(fo.reg, t) * state_pack(gd, sd)

    y0 = state_pack(chans, sigma)
    if aam:
        y0 = np.concatenate([y0, [sigma_inf + 0j]])
    y, ts, rej = ode_solve(f, y0, flow_t(fo.reg, lam_i), flow_t(fo.reg, lam_f), steps,
                           fo.adaptive, fo.atol, fo.rtol, fo.max_steps)
    info["lambdas"] = [flow_lambda(fo.reg, t) for t in ts]
    info["rejected"] = rej
    if aam:
        info["sigma_inf"] = float(y[-1].real)
        y = y[:-1]
    ch, sg = state_unpack(y, n)
    return ch, sg, info


def regrid(src: Grid, dst: Grid, chans=None, sigma=None):
    """Classes and self-energy carried from grid src onto grid dst by the lookup every evaluation
    uses (Sec. Interpolation routines: linear in each auxiliary variable, zero outside the
    extent): each class of channel r is read by vertex_eval in r's own parametrisation at the
    nodes of dst; sigma [n][4] is interpolated on src's auxiliary variable node by node.
    Returns (chans, sigma) on dst (None where not given)."""
    v = dst.nodes()
    nd = dst.n
    out_ch = None
    if chans is not None:
        out_ch = []
        for r, ch in enumerate(chans):
            chs = [Channel(0.0), Channel(0.0), Channel(0.0)]
            chs[r] = Channel(1.0, ch.K1, ch.K2, ch.K2p, ch.K3)
            V = Vertex(src, 0.0, chs)
            new = {}
            if ch.K1 is not None:
                pts = np.stack([v, 0 * v, 0 * v], 1)
                new["K1"] = np.transpose(vertex_eval(V, r, pts, P_K1), (1, 0, 2)).copy()
            W, X = np.meshgrid(v, v, indexing="ij")
            if ch.K2 is not None:
                pts = np.stack([W.ravel(), X.ravel(), 0 * W.ravel()], 1)
                new["K2"] = np.transpose(vertex_eval(V, r, pts, P_K2).reshape(nd, nd, 2, 16), (2, 0, 1, 3)).copy()
            if ch.K2p is not None:
                pts = np.stack([W.ravel(), 0 * W.ravel(), X.ravel()], 1)
                new["K2p"] = np.transpose(vertex_eval(V, r, pts, P_K2P).reshape(nd, nd, 2, 16), (2, 0, 1, 3)).copy()
            if ch.K3 is not None:
                W3, X3, Y3 = np.meshgrid(v, v, v, indexing="ij")
                pts = np.stack([W3.ravel(), X3.ravel(), Y3.ravel()], 1)
                new["K3"] = np.transpose(vertex_eval(V, r, pts, P_K3).reshape(nd, nd, nd, 2, 16),
                                         (3, 0, 1, 2, 4)).copy()
            out_ch.append(Channel(ch.coef, new.get("K1"), new.get("K2"), new.get("K2p"), new.get("K3")))
    out_sig = None
    if sigma is not None:
        sigma = np.asarray(sigma)
        out_sig = np.zeros((nd, 4), dtype=np.complex128)
        i0, t = C.c_int(), C.c_double()
        for i in range(nd):
            if lib().oracle_grid_locate(src.n, src.L, src.a, src.map, v[i], C.byref(i0), C.byref(t)):
                out_sig[i] = (1.0 - t.value) * sigma[i0.value] + t.value * sigma[i0.value + 1]
    return out_ch, out_sig
