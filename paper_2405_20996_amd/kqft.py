"""Thin ctypes binding of libkqft.so (include/kqft.h): argument marshalling only.

Every step of the computation runs in the HIP library; torch supplies device memory
and streams.  There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkqft.so")

CH_A, CH_P, CH_T = 0, 1, 2
FP64, SPLIT_FP32 = 0, 1
PI_GG, PI_DOT = 0, 1
REG_DELTA, REG_U, REG_T, REG_NU = 0, 1, 2, 3
LINE_G, LINE_S, LINE_GSG = 0, 1, 2
ENOCONV = -5
K1, K2, K2P, K3, KALL = 1, 2, 4, 8, 15
QUAD_TAN_FINITE, QUAD_TAN_INFINITE = 0, 1
GRID_TAN, GRID_ALGEBRAIC = 0, 1
CLASSES = ("K1", "K2", "K2p", "K3")


class KqftGrid(C.Structure):
    _fields_ = [("n", C.c_int), ("L", C.c_double), ("a", C.c_double), ("map", C.c_int)]


class KqftQuad(C.Structure):
    _fields_ = [("n", C.c_int), ("map", C.c_int), ("L", C.c_double), ("a", C.c_double)]


class KqftChvert(C.Structure):
    _fields_ = [("coef", C.c_double), ("K1", C.c_void_p), ("K2", C.c_void_p), ("K2p", C.c_void_p),
                ("K3", C.c_void_p)]


class KqftVertex(C.Structure):
    _fields_ = [("r0", C.c_double), ("grid", KqftGrid), ("ch", KqftChvert * 3)]


class KqftMGrid(C.Structure):
    _fields_ = [("M", C.c_int), ("N", C.c_int), ("T", C.c_double)]


class KqftMVertex(C.Structure):
    _fields_ = [("grid", KqftMGrid), ("U", C.c_double), ("ch", KqftChvert * 3)]


class KqftMProp(C.Structure):
    _fields_ = [("Delta", C.c_double), ("sigma", C.c_void_p), ("sigma_N", C.c_int), ("dsigma", C.c_void_p),
                ("reg", C.c_int), ("lam", C.c_double)]


class KqftPropagator(C.Structure):
    _fields_ = [("Delta", C.c_double), ("T", C.c_double), ("eps", C.c_double), ("sgrid", KqftGrid),
                ("SigR", C.c_void_p), ("SigK", C.c_void_p), ("reg", C.c_int), ("lam", C.c_double),
                ("dSigR", C.c_void_p), ("dSigK", C.c_void_p), ("deps", C.c_double)]


class KqftFlowOpts(C.Structure):
    _fields_ = [("reg", C.c_int), ("Delta", C.c_double), ("katanin", C.c_int), ("se_iterations", C.c_int),
                ("se_tol_abs", C.c_double), ("se_tol_rel", C.c_double), ("se_anderson", C.c_int), ("adaptive", C.c_int),
                ("ode_tol_abs", C.c_double), ("ode_tol_rel", C.c_double), ("max_steps", C.c_int),
                ("asymmetric", C.c_int), ("eps_d", C.c_double), ("sigma_inf", C.c_double)]


class KqftParquetOpts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("max_iterations", C.c_int), ("tol", C.c_double),
                ("anderson_depth", C.c_int), ("reduce_alpha", C.c_int), ("alpha_min", C.c_double),
                ("hartree", C.c_int), ("eps_d", C.c_double), ("q_hartree", KqftQuad), ("hartree_tol", C.c_double),
                ("sde_forms", C.c_int)]


class KqftAdaptInfo(C.Structure):
    _fields_ = [("intervals", C.c_longlong), ("generations", C.c_int), ("evaluations", C.c_longlong)]


class KqftFlowInfo(C.Structure):
    _fields_ = [("accepted", C.c_int), ("rejected", C.c_int), ("rhs_evaluations", C.c_int),
                ("se_iterations", C.c_int), ("sigma_inf", C.c_double)]


class KqftChout(C.Structure):
    _fields_ = [("K1", C.c_void_p), ("K2", C.c_void_p), ("K2p", C.c_void_p), ("K3", C.c_void_p)]


class KqftOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("class_mask", C.c_int), ("beta", C.c_int), ("omega_batch", C.c_int),
                ("overlap", C.c_int)]


_lib = None
_ctx = {}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        _lib = C.CDLL(LIB_PATH)
        P = C.POINTER
        _lib.kqft_ctx_create.argtypes = [P(C.c_void_p), C.c_int]
        _lib.kqft_ctx_destroy.argtypes = [C.c_void_p]
        _lib.kqft_last_error.restype = C.c_char_p
        _lib.kqft_ctx_profile.argtypes = [C.c_void_p, C.c_int]
        _lib.kqft_ctx_profile_read.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.kqft_bubble_workspace.restype = C.c_size_t
        _lib.kqft_bubble_workspace.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        _lib.kqft_bubble.argtypes = [C.c_void_p, C.c_int, P(KqftVertex), P(KqftVertex), P(KqftPropagator), C.c_int,
                                     P(KqftQuad), P(KqftOpts), P(KqftChout), C.c_void_p]
        _lib.kqft_sde.argtypes = [C.c_void_p, P(KqftVertex), P(KqftPropagator), P(KqftQuad), P(KqftQuad),
                                  P(KqftOpts), C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.kqft_mloop_step.argtypes = [C.c_void_p, C.c_int, P(KqftVertex), P(KqftPropagator), P(KqftQuad), C.c_int,
                                         P(KqftOpts), P(KqftChout), C.c_void_p]
        _lib.kqft_sde_adjoint.argtypes = [C.c_void_p, P(KqftVertex), P(KqftPropagator), P(KqftQuad), P(KqftQuad),
                                          P(KqftOpts), C.c_void_p, P(KqftChout), C.c_void_p, C.c_void_p]
        _lib.kqft_bubble_adjoint.argtypes = [C.c_void_p, C.c_int, P(KqftVertex), P(KqftVertex), P(KqftPropagator),
                                             C.c_int, P(KqftQuad), P(KqftOpts), P(KqftChout), P(KqftChout),
                                             P(KqftChout), C.c_void_p, C.c_void_p]
        _lib.kqft_mloop_adjoint.argtypes = [C.c_void_p, P(KqftVertex), P(KqftPropagator), P(KqftQuad), C.c_int,
                                            P(KqftOpts), P(KqftChout), P(KqftChout), C.c_void_p, C.c_void_p]
        _lib.kqft_mloop_jvp.argtypes = [C.c_void_p, P(KqftVertex), P(KqftVertex), P(KqftPropagator), P(KqftQuad),
                                        C.c_int, P(KqftOpts), P(KqftChout), P(KqftChout), C.c_void_p]
        _lib.kqft_workspace_bytes.argtypes = [P(C.c_size_t), P(C.c_size_t)]
        _lib.kqft_workspace_reset_peak.argtypes = []
        _lib.kqft_bubble_tune.argtypes = [C.c_void_p, C.c_int, P(KqftVertex), P(KqftVertex), P(KqftPropagator),
                                          C.c_int, P(KqftQuad), P(KqftOpts), P(KqftChout), C.c_size_t,
                                          P(C.c_int), P(C.c_double), C.c_void_p]
        _lib.kqft_chi_noalloc.argtypes = [C.c_int, P(KqftVertex), P(KqftPropagator), P(KqftQuad), C.c_void_p,
                                          C.c_void_p]
        _lib.kqft_chi.argtypes = [C.c_void_p, C.c_int, P(KqftVertex), P(KqftPropagator), P(KqftQuad), C.c_void_p,
                                  C.c_void_p]
        _lib.kqft_bubble_matsubara.argtypes = [C.c_void_p, C.c_int, P(KqftMVertex), P(KqftMVertex), P(KqftMProp),
                                               C.c_int, C.c_int, C.c_int, P(KqftChout), C.c_void_p]
        _lib.kqft_regrid.argtypes = [C.c_void_p, P(KqftGrid), P(KqftGrid), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]
        _lib.kqft_chi_matsubara.argtypes = [C.c_void_p, C.c_int, P(KqftMVertex), P(KqftMProp), C.c_int, C.c_void_p,
                                            C.c_void_p]
        _lib.kqft_loop_matsubara.argtypes = [C.c_void_p, P(KqftMVertex), P(KqftMProp), C.c_int, C.c_int, C.c_void_p,
                                             C.c_void_p]
        _lib.kqft_mfrg_flow_matsubara.argtypes = [C.c_void_p, P(KqftMGrid), C.c_double, C.c_double, C.c_double,
                                                  C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                                  C.c_double, C.c_int, C.c_double, C.c_double, C.c_int,
                                                  P(KqftChout), C.c_void_p, C.c_void_p, P(KqftFlowInfo), C.c_void_p]
        _lib.kqft_sde_matsubara.argtypes = [C.c_void_p, P(KqftMVertex), P(KqftMProp), C.c_int, C.c_int, C.c_void_p,
                                            C.c_void_p]
        _lib.kqft_parquet_solve_matsubara.argtypes = [C.c_void_p, P(KqftMGrid), C.c_double, C.c_double, C.c_int,
                                                      C.c_int, P(KqftParquetOpts), P(KqftChout), C.c_void_p,
                                                      P(C.c_double), P(C.c_int), C.c_void_p]
        _lib.kqft_loop.argtypes = [C.c_void_p, P(KqftVertex), P(KqftPropagator), C.c_int, P(KqftQuad), C.c_void_p,
                                   C.c_void_p]
        _lib.kqft_mfrg_flow.argtypes = [C.c_void_p, P(KqftGrid), C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_int, C.c_int, P(KqftQuad), P(KqftQuad), P(KqftOpts), P(KqftFlowOpts),
                                        P(KqftChout), C.c_void_p, C.c_void_p, P(KqftFlowInfo), C.c_void_p]
        _lib.kqft_parquet_iteration.argtypes = [C.c_void_p, P(KqftVertex), P(KqftPropagator), P(KqftQuad),
                                                P(KqftQuad), P(KqftOpts), P(KqftChout), C.c_void_p, C.c_void_p]
        _lib.kqft_bubble_adaptive.argtypes = [C.c_void_p, C.c_int, P(KqftVertex), P(KqftVertex), P(KqftPropagator),
                                              C.c_int, P(KqftQuad), C.c_double, P(KqftOpts), P(KqftChout),
                                              P(KqftAdaptInfo), C.c_void_p]
        _lib.kqft_hartree.argtypes = [C.c_void_p, C.c_double, C.c_double, P(KqftPropagator), P(KqftQuad), C.c_int,
                                      C.c_double, P(C.c_double), P(C.c_int), C.c_void_p]
        _lib.kqft_parquet_solve.argtypes = [C.c_void_p, P(KqftGrid), C.c_double, C.c_double, C.c_double,
                                            P(KqftQuad), P(KqftQuad), P(KqftOpts), P(KqftParquetOpts),
                                            P(KqftChout), C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_int),
                                            C.c_void_p]
    return _lib


def exported_symbols() -> list:
    names = ["kqft_ctx_create", "kqft_ctx_destroy", "kqft_last_error", "kqft_ctx_profile", "kqft_ctx_profile_read",
             "kqft_bubble_workspace", "kqft_bubble",
             "kqft_sde", "kqft_mloop_step", "kqft_bubble_adjoint", "kqft_sde_adjoint", "kqft_mloop_adjoint",
             "kqft_mloop_jvp", "kqft_workspace_bytes", "kqft_workspace_reset_peak", "kqft_chi_noalloc",
             "kqft_bubble_tune"]
    L = lib()
    return [n for n in names if hasattr(L, n)]


class KqftError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        raise KqftError(f"kqft error {rc}: {lib().kqft_last_error().decode()}")


def ctx(device: Optional[int] = None):
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _ctx:
        h = C.c_void_p()
        _check(lib().kqft_ctx_create(C.byref(h), dev))
        _ctx[dev] = h
    return _ctx[dev]


def _stream(stream) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def profile(enable: bool = True):
    _check(lib().kqft_ctx_profile(ctx(), int(enable)))


def profile_read():
    """Per kernel kind (pi, gather, gemm, reductions): (summed ms, launches), then cleared."""
    ms = (C.c_double * 4)()
    n = (C.c_int * 4)()
    _check(lib().kqft_ctx_profile_read(ctx(), ms, n))
    return {k: (ms[i], n[i]) for i, k in enumerate(("pi", "gather", "gemm", "reduce"))}


# ------------------------------------------------------------------ data model
@dataclass
class Grid:
    n: int
    L: float = 20.0
    a: float = 1.0
    map: int = GRID_TAN

    def c(self) -> KqftGrid:
        return KqftGrid(self.n, self.L, self.a, self.map)


@dataclass
class Quad:
    n: int
    map: int = QUAD_TAN_FINITE
    L: float = 20.0
    a: float = 1.0

    def c(self) -> KqftQuad:
        return KqftQuad(self.n, self.map, self.L, self.a)


def class_shape(name: str, n: int) -> tuple:
    return {"K1": (2, n, 16), "K2": (2, n, n, 16), "K2p": (2, n, n, 16), "K3": (2, n, n, n, 16)}[name]


def _ptr(t: Optional[torch.Tensor], shape=None, what="") -> Optional[int]:
    if t is None:
        return None
    if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: needs a contiguous complex128 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: shape {tuple(t.shape)} != {tuple(shape)}")
    return t.data_ptr()


@dataclass
class Channel:
    coef: float = 1.0
    K1: Optional[torch.Tensor] = None
    K2: Optional[torch.Tensor] = None
    K2p: Optional[torch.Tensor] = None
    K3: Optional[torch.Tensor] = None


@dataclass
class Vertex:
    """Gamma = Gamma_0(r0) + sum_r coef_r gamma_r (class tensors complex128 on the device)."""
    grid: Grid
    r0: float = 0.0
    ch: list = field(default_factory=lambda: [Channel(0.0), Channel(0.0), Channel(0.0)])

    def c(self) -> KqftVertex:
        v = KqftVertex()
        v.r0 = self.r0
        v.grid = self.grid.c()
        for r in range(3):
            chn = self.ch[r]
            v.ch[r].coef = chn.coef
            for name in CLASSES:
                setattr(v.ch[r], name, _ptr(getattr(chn, name), class_shape(name, self.grid.n), f"ch{r}.{name}"))
        return v


@dataclass
class Propagator:
    """G^R = 1/(G_0^{-1,R} - Sigma^R) with the regulator `reg` (lam for REG_U / REG_NU);
    dSigR/dSigK: optional Sigma_dot (Katanin substitution, G Sigma_dot G line); deps: a real
    constant added to Sigma_dot^R (the flow of the level)."""
    Delta: float = 1.0
    T: float = 0.1
    eps: float = 0.0
    sigma_grid: Optional[Grid] = None
    SigR: Optional[torch.Tensor] = None
    SigK: Optional[torch.Tensor] = None
    reg: int = REG_DELTA
    lam: float = 1.0
    dSigR: Optional[torch.Tensor] = None
    dSigK: Optional[torch.Tensor] = None
    deps: float = 0.0

    def c(self) -> KqftPropagator:
        g = (self.sigma_grid or Grid(2, 1.0, 1.0)).c()
        n = self.sigma_grid.n if self.sigma_grid else None
        sh = (n,) if n else None
        return KqftPropagator(self.Delta, self.T, self.eps, g, _ptr(self.SigR, sh, "SigR"), _ptr(self.SigK, sh, "SigK"),
                              self.reg, self.lam, _ptr(self.dSigR, sh, "dSigR"), _ptr(self.dSigK, sh, "dSigK"),
                              self.deps)


@dataclass
class FlowOptions:
    """kqft_flow_opts: regulator, Katanin substitution, self-energy corrections, ODE method;
    eps_d (not None): the asymmetric model with level eps_d + Sigma_inf, starting at sigma_inf."""
    reg: int = REG_DELTA
    Delta: float = 1.0
    katanin: bool = True
    se_iterations: int = 0
    se_atol: float = 1e-9
    se_rtol: float = 1e-5
    se_anderson: int = 0
    adaptive: bool = False
    atol: float = 1e-8
    rtol: float = 1e-5
    max_steps: int = 200
    eps_d: Optional[float] = None
    sigma_inf: float = 0.0

    def c(self) -> KqftFlowOpts:
        return KqftFlowOpts(self.reg, self.Delta, int(self.katanin), self.se_iterations, self.se_atol, self.se_rtol,
                            self.se_anderson, int(self.adaptive), self.atol, self.rtol, self.max_steps,
                            int(self.eps_d is not None), self.eps_d or 0.0, self.sigma_inf)


def _opts(precision, class_mask, beta, omega_batch, overlap=0) -> KqftOpts:
    return KqftOpts(precision, class_mask, beta, omega_batch, overlap)


@dataclass
class MGrid:
    """Matsubara boxes: bosonic m in [-M, M], fermionic n in [-N, N), temperature T."""
    M: int
    N: int
    T: float

    def c(self) -> KqftMGrid:
        return KqftMGrid(self.M, self.N, self.T)

    def shape(self, name: str) -> tuple:
        nb, nf = 2 * self.M + 1, 2 * self.N
        return {"K1": (2, nb), "K2": (2, nb, nf), "K2p": (2, nb, nf), "K3": (2, nb, nf, nf)}[name]


@dataclass
class MVertex:
    """Matsubara vertex Gamma_0 (X0 = -U, Y0 = +U) + sum_r coef_r gamma_r (device tensors)."""
    grid: MGrid
    U: float = 0.0
    ch: list = field(default_factory=lambda: [Channel(0.0), Channel(0.0), Channel(0.0)])

    def c(self) -> KqftMVertex:
        v = KqftMVertex()
        v.grid = self.grid.c()
        v.U = self.U
        for r in range(3):
            chn = self.ch[r]
            v.ch[r].coef = chn.coef
            for name in CLASSES:
                setattr(v.ch[r], name, _ptr(getattr(chn, name), self.grid.shape(name), f"ch{r}.{name}"))
        return v


def alloc_channel(n: int, device=None, zero: bool = True) -> Channel:
    dev = device or torch.device("cuda", torch.cuda.current_device())
    f = torch.zeros if zero else torch.empty
    return Channel(1.0, *[f(class_shape(c, n), dtype=torch.complex128, device=dev) for c in CLASSES])


def _chout(chn: Channel, n: int) -> KqftChout:
    return KqftChout(*[_ptr(getattr(chn, c), class_shape(c, n), f"out.{c}") for c in CLASSES])


def _chout_opt(chn: Optional[Channel], n: int) -> KqftChout:
    if chn is None:
        return KqftChout(None, None, None, None)
    return _chout(chn, n)


# ------------------------------------------------------------------ entry points
def bubble(channel: int, left: Vertex, right: Vertex, G: Propagator, q: Quad, pi_kind: int = PI_GG,
           precision: int = FP64, class_mask: int = KALL, beta: int = 0, omega_batch: int = 0,
           out: Optional[Channel] = None, stream=None, overlap: bool = False) -> Channel:
    n = left.grid.n
    if out is None:
        out = alloc_channel(n)
    lc, rc, gc, qc = left.c(), right.c(), G.c(), q.c()
    oc = _chout(out, n)
    _check(lib().kqft_bubble(ctx(), channel, C.byref(lc), C.byref(rc), C.byref(gc), pi_kind, C.byref(qc),
                             C.byref(_opts(precision, class_mask, beta, omega_batch, int(overlap))), C.byref(oc),
                             _stream(stream)))
    return out


def sde(gamma: Vertex, G: Propagator, q_bubble: Quad, q_loop: Quad, precision: int = FP64, with_chi: bool = True,
        omega_batch: int = 0, stream=None):
    n = gamma.grid.n
    dev = torch.device("cuda", torch.cuda.current_device())
    sigma = torch.zeros((n, 4), dtype=torch.complex128, device=dev)
    chi = torch.zeros((2, n, 16), dtype=torch.complex128, device=dev) if with_chi else None
    vc, gc, qb, ql = gamma.c(), G.c(), q_bubble.c(), q_loop.c()
    _check(lib().kqft_sde(ctx(), C.byref(vc), C.byref(gc), C.byref(qb), C.byref(ql),
                          C.byref(_opts(precision, KALL, 0, omega_batch)), C.c_void_p(sigma.data_ptr()),
                          C.c_void_p(chi.data_ptr() if chi is not None else None), _stream(stream)))
    return sigma, chi


def chi(channel: int, gamma: Vertex, G: Propagator, q: Quad, stream=None) -> torch.Tensor:
    """Pair-space susceptibility of one channel: [2 (spin combinations), n, 16] complex."""
    n = gamma.grid.n
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.zeros((2, n, 16), dtype=torch.complex128, device=dev)
    vc, gc, qc = gamma.c(), G.c(), q.c()
    _check(lib().kqft_chi(ctx(), channel, C.byref(vc), C.byref(gc), C.byref(qc), C.c_void_p(out.data_ptr()),
                          _stream(stream)))
    return out


def _mprop(Delta: float, sigma: Optional[torch.Tensor], dsigma: Optional[torch.Tensor], reg: int = 0,
           lam: float = 1.0) -> KqftMProp:
    ref = sigma if sigma is not None else dsigma
    ns = 0 if ref is None else ref.shape[0] // 2
    for t in (sigma, dsigma):
        if t is not None and t.shape[0] != 2 * ns:
            raise ValueError("sigma and dsigma need the same even length 2 Ns")
    return KqftMProp(Delta, _ptr(sigma, None, "sigma"), ns, _ptr(dsigma, None, "dsigma"), reg, lam)


def bubble_matsubara(channel: int, left: MVertex, right: MVertex, Delta: float, Nq: int,
                     sigma: Optional[torch.Tensor] = None, out: Optional[Channel] = None, pi_kind: int = PI_GG,
                     dsigma: Optional[torch.Tensor] = None, tails: bool = False, reg: int = 0, lam: float = 1.0,
                     stream=None) -> Channel:
    """B_channel(left, right) in the Matsubara formalism (sum over 2 Nq fermionic frequencies about
    the bubble's centre); sigma: Sigma(i nu_n) on n in [-Ns, Ns) (length 2 Ns) or None; pi_kind
    PI_DOT: Pi_dot along S = dG/dDelta (+ G dsigma G); tails: the analytic tails beyond the window."""
    g = left.grid
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = Channel(1.0, *[torch.zeros(g.shape(c), dtype=torch.complex128, device=dev) for c in CLASSES])
    gp = _mprop(Delta, sigma, dsigma, reg, lam)
    oc = KqftChout(*[_ptr(getattr(out, c), g.shape(c), f"out.{c}") for c in CLASSES])
    lc, rc = left.c(), right.c()
    _check(lib().kqft_bubble_matsubara(ctx(), channel, C.byref(lc), C.byref(rc), C.byref(gp), pi_kind, Nq,
                                       int(tails), C.byref(oc), _stream(stream)))
    return out


def regrid(src: Grid, dst: Grid, gamma: Optional[Sequence[Channel]] = None, sigma: Optional[torch.Tensor] = None,
           stream=None):
    """The channels' classes (coefficients kept) and the self-energy [n][4] carried from grid src onto
    grid dst.  Returns (channels, sigma) on dst (None where not given)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    gin = gout = None
    new = None
    keep = []
    if gamma is not None:
        new = [Channel(c.coef, *[None if getattr(c, x) is None else
                                 torch.zeros(class_shape(x, dst.n), dtype=torch.complex128, device=dev)
                                 for x in CLASSES]) for c in gamma]
        gin = (KqftChout * 3)(*[_chout(c, src.n) for c in gamma])
        gout = (KqftChout * 3)(*[_chout(c, dst.n) for c in new])
        keep += [gin, gout]
    sig = None
    if sigma is not None:
        _ptr(sigma, (src.n, 4), "sigma")
        sig = torch.zeros((dst.n, 4), dtype=torch.complex128, device=dev)
    sc, dc = src.c(), dst.c()
    _check(lib().kqft_regrid(ctx(), C.byref(sc), C.byref(dc), C.cast(gin, C.c_void_p) if gin else None,
                             C.c_void_p(sigma.data_ptr()) if sigma is not None else None,
                             C.cast(gout, C.c_void_p) if gout else None,
                             C.c_void_p(sig.data_ptr()) if sig is not None else None, _stream(stream)))
    return new, sig


def chi_matsubara(channel: int, gamma: MVertex, Delta: float, Nq: int, sigma: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Susceptibility of one channel in the Matsubara formalism: [2 (combinations), 2M + 1]."""
    g = gamma.grid
    out = torch.zeros((2, 2 * g.M + 1), dtype=torch.complex128,
                      device=torch.device("cuda", torch.cuda.current_device()))
    gp = _mprop(Delta, sigma, None)
    vc = gamma.c()
    _check(lib().kqft_chi_matsubara(ctx(), channel, C.byref(vc), C.byref(gp), Nq, C.c_void_p(out.data_ptr()),
                                    _stream(stream)))
    return out


def loop_matsubara(gamma: MVertex, Delta: float, Nl: int, kind: int = LINE_G, sigma: Optional[torch.Tensor] = None,
                   dsigma: Optional[torch.Tensor] = None, reg: int = 0, lam: float = 1.0,
                   stream=None) -> torch.Tensor:
    """L(Gamma, X)(i nu_n), n in [-N, N), X = G, S (+ G dsigma G) or G dsigma G."""
    g = gamma.grid
    out = torch.zeros(2 * g.N, dtype=torch.complex128, device=torch.device("cuda", torch.cuda.current_device()))
    gp = _mprop(Delta, sigma, dsigma, reg, lam)
    vc = gamma.c()
    _check(lib().kqft_loop_matsubara(ctx(), C.byref(vc), C.byref(gp), kind, Nl, C.c_void_p(out.data_ptr()),
                                     _stream(stream)))
    return out


def mfrg_flow_matsubara(grid: MGrid, U: float, lam_i: float, lam_f: float, steps: int, nloops: int, Nq: int, Nl: int,
                        gamma: Sequence[Channel], sigma: torch.Tensor, katanin: bool = True, se_iterations: int = 0,
                        se_atol: float = 1e-9, se_rtol: float = 1e-5, adaptive: bool = False, atol: float = 1e-8,
                        rtol: float = 1e-5, max_steps: int = 200, reg: int = 0, Delta: float = 1.0, stream=None):
    """The Matsubara hybridization flow of the state (gamma[3], sigma [2N]) from lam_i to lam_f,
    in place (classical RK4, or Cash-Karp step control with adaptive).  Returns (gamma, sigma,
    info) with info the accepted Delta values and the step counts."""
    D = (KqftChout * 3)(*[KqftChout(*[_ptr(getattr(c, x), grid.shape(x), f"gamma.{x}") for x in CLASSES])
                          for c in gamma])
    _ptr(sigma, (2 * grid.N,), "sigma")
    gc = grid.c()
    lams = (C.c_double * ((max_steps if adaptive else steps) + 1))()
    inf = KqftFlowInfo()
    _check(lib().kqft_mfrg_flow_matsubara(ctx(), C.byref(gc), C.c_double(U), C.c_double(lam_i), C.c_double(lam_f),
                                          reg, C.c_double(Delta), steps, nloops, Nq, Nl, int(katanin), se_iterations, C.c_double(se_atol),
                                          C.c_double(se_rtol), int(adaptive), C.c_double(atol), C.c_double(rtol),
                                          max_steps, D, C.c_void_p(sigma.data_ptr()), lams, C.byref(inf),
                                          _stream(stream)))
    info = {"lambdas": list(lams[:inf.accepted + 1]), "accepted": inf.accepted, "rejected": inf.rejected,
            "rhs": inf.rhs_evaluations, "se_iterations": inf.se_iterations}
    return gamma, sigma, info


def sde_matsubara(gamma: MVertex, Delta: float, Nq: int, Nl: int, sigma: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Sigma(i nu_n), n in [-N, N), from the Matsubara SDE (a-channel form) of gamma."""
    g = gamma.grid
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.zeros(2 * g.N, dtype=torch.complex128, device=dev)
    gp = _mprop(Delta, sigma, None)
    vc = gamma.c()
    _check(lib().kqft_sde_matsubara(ctx(), C.byref(vc), C.byref(gp), Nq, Nl, C.c_void_p(out.data_ptr()),
                                    _stream(stream)))
    return out


def parquet_solve_matsubara(grid: MGrid, U: float, Delta: float, Nq: int, Nl: int, alpha: float = 0.5,
                            max_iterations: int = 20, tol: float = 0.0, depth: int = 0, reduce_alpha: bool = False,
                            alpha_min: float = 0.01, stream=None):
    """Matsubara parquet solver from the PT2 state; returns (channels, Sigma [2N], residuals)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    outs = [Channel(1.0, *[torch.zeros(grid.shape(c), dtype=torch.complex128, device=dev) for c in CLASSES])
            for _ in range(3)]
    sigma = torch.zeros(2 * grid.N, dtype=torch.complex128, device=dev)
    res = (C.c_double * max_iterations)()
    its = C.c_int(0)
    D = (KqftChout * 3)(*[KqftChout(*[_ptr(getattr(o, c), grid.shape(c), f"out.{c}") for c in CLASSES])
                          for o in outs])
    po = KqftParquetOpts(alpha, max_iterations, tol, depth, int(reduce_alpha), alpha_min, 0, 0.0,
                         KqftQuad(1, QUAD_TAN_INFINITE, 0.0, 1.0), 1e-12, 1)
    gc = grid.c()
    _check(lib().kqft_parquet_solve_matsubara(ctx(), C.byref(gc), C.c_double(U), C.c_double(Delta), Nq, Nl,
                                              C.byref(po), D, C.c_void_p(sigma.data_ptr()), res, C.byref(its),
                                              _stream(stream)))
    return outs, sigma, [res[i] for i in range(its.value)]


def mloop_step(gammas: Sequence[Vertex], Gs: Sequence[Propagator], qs: Sequence[Quad], nloops: int,
               precision: int = FP64, omega_batch: int = 0, stream=None) -> list:
    """Returns out[p][l][r] (Channel): order-(l+1) insertions of point p in channel r."""
    npts = len(gammas)
    outs = [[[alloc_channel(g.grid.n) for _ in range(3)] for _ in range(nloops)] for g in gammas]
    V = (KqftVertex * npts)(*[g.c() for g in gammas])
    P = (KqftPropagator * npts)(*[g.c() for g in Gs])
    Q = (KqftQuad * npts)(*[q.c() for q in qs])
    D = (KqftChout * (npts * nloops * 3))(*[_chout(outs[p][l][r], gammas[p].grid.n)
                                             for p in range(npts) for l in range(nloops) for r in range(3)])
    _check(lib().kqft_mloop_step(ctx(), npts, V, P, Q, nloops, C.byref(_opts(precision, KALL, 0, omega_batch)), D,
                                 _stream(stream)))
    return outs


def loop(gamma: Vertex, G: Propagator, q: Quad, kind: int = LINE_G, stream=None) -> torch.Tensor:
    """L(Gamma, X) [n][4] (no overall sign), X = G, S (+ G Sigma_dot G) or G Sigma_dot G by kind;
    the one-loop self-energy flow is -loop(Gamma, G, q, LINE_S)."""
    n = gamma.grid.n
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.zeros((n, 4), dtype=torch.complex128, device=dev)
    vc, gc, qc = gamma.c(), G.c(), q.c()
    _check(lib().kqft_loop(ctx(), C.byref(vc), C.byref(gc), kind, C.byref(qc), C.c_void_p(out.data_ptr()),
                           _stream(stream)))
    return out


def mfrg_flow(grid: Grid, U: float, T: float, lam_i: float, lam_f: float, steps: int, nloops: int,
              q_bubble: Quad, q_loop: Quad, gamma: Sequence[Channel], sigma: torch.Tensor,
              flow: Optional[FlowOptions] = None, precision: int = FP64, stream=None):
    """Flow of the state (gamma[3] Channels, sigma [n][4]) from lam_i to lam_f, in place.
    Returns (gamma, sigma, info) with info the accepted flow parameters and step counts (and
    sigma_inf, the final asymptotic value of the self-energy, for the asymmetric model)."""
    n = grid.n
    fo = flow or FlowOptions()
    D = (KqftChout * 3)(*[_chout(c, n) for c in gamma])
    _ptr(sigma, (n, 4), "sigma")
    gc, qb, ql = grid.c(), q_bubble.c(), q_loop.c()
    cap = (fo.max_steps if fo.adaptive else steps) + 1
    lams = (C.c_double * cap)()
    inf = KqftFlowInfo()
    rc = lib().kqft_mfrg_flow(ctx(), C.byref(gc), C.c_double(U), C.c_double(T), C.c_double(lam_i),
                              C.c_double(lam_f), steps, nloops, C.byref(qb), C.byref(ql),
                              C.byref(_opts(precision, KALL, 0, 0)), C.byref(fo.c()), D, C.c_void_p(sigma.data_ptr()),
                              lams, C.byref(inf), _stream(stream))
    _check(rc)
    info = {"lambdas": list(lams[:inf.accepted + 1]), "accepted": inf.accepted, "rejected": inf.rejected,
            "rhs": inf.rhs_evaluations, "se_iterations": inf.se_iterations, "sigma_inf": inf.sigma_inf}
    return gamma, sigma, info


def parquet_iteration(gamma: Vertex, G: Propagator, q_bubble: Quad, q_loop: Quad, precision: int = FP64,
                      stream=None):
    """(gamma_a', gamma_p', gamma_t') as Channels and Sigma' [n][4]: the symmetrized BSEs and the SDE."""
    n = gamma.grid.n
    outs = [alloc_channel(n) for _ in range(3)]
    dev = torch.device("cuda", torch.cuda.current_device())
    sigma = torch.zeros((n, 4), dtype=torch.complex128, device=dev)
    D = (KqftChout * 3)(*[_chout(o, n) for o in outs])
    vc, gc, qb, ql = gamma.c(), G.c(), q_bubble.c(), q_loop.c()
    _check(lib().kqft_parquet_iteration(ctx(), C.byref(vc), C.byref(gc), C.byref(qb), C.byref(ql),
                                        C.byref(_opts(precision, KALL, 0, 0)), D, C.c_void_p(sigma.data_ptr()),
                                        _stream(stream)))
    return outs, sigma


def bubble_adaptive(channel: int, left: Vertex, right: Vertex, G: Propagator, q: Quad, eps: float = 1e-5,
                    pi_kind: int = PI_GG, class_mask: int = KALL, out: Optional[Channel] = None, stream=None):
    """B_channel(left, right) with adaptive Gauss-Lobatto-Kronrod integration per output over q's
    finite tangent map; returns (Channel of outputs, info dict)."""
    n = left.grid.n
    if out is None:
        out = alloc_channel(n, zero=False)
    lc, rc_, gc, qc = left.c(), right.c(), G.c(), q.c()
    co = _chout_opt(out, n)
    inf = KqftAdaptInfo()
    _check(lib().kqft_bubble_adaptive(ctx(), channel, C.byref(lc), C.byref(rc_), C.byref(gc), pi_kind, C.byref(qc),
                                      C.c_double(eps), C.byref(_opts(FP64, class_mask, 0, 0)), C.byref(co),
                                      C.byref(inf), _stream(stream)))
    return out, {"intervals": inf.intervals, "generations": inf.generations, "evaluations": inf.evaluations}


def hartree(U: float, eps_d: float, G: Propagator, q: Quad, self_consistent: bool = True, tol: float = 1e-12,
            sigma_H: float = 0.0, stream=None):
    """Hartree term Sigma_H = U <n> of the level eps_d (one shot from sigma_H, or self-consistent);
    returns (Sigma_H, evaluations of <n>)."""
    val = C.c_double(sigma_H)
    its = C.c_int(0)
    gc, qc = G.c(), q.c()
    _check(lib().kqft_hartree(ctx(), C.c_double(U), C.c_double(eps_d), C.byref(gc), C.byref(qc),
                              int(self_consistent), C.c_double(tol), C.byref(val), C.byref(its), _stream(stream)))
    return val.value, its.value


def parquet_solve(grid: Grid, U: float, Delta: float, T: float, q_bubble: Quad, q_loop: Quad, alpha: float = 0.5,
                  max_iterations: int = 20, tol: float = 0.0, precision: int = FP64, depth: int = 0,
                  reduce_alpha: bool = False, alpha_min: float = 0.01, eps_d: Optional[float] = None,
                  q_hartree: Optional[Quad] = None, hartree_tol: float = 1e-12, sde_forms: int = 1, stream=None):
    """Parquet solver from the PT2 state with linear mixing or Anderson acceleration of the
    given depth; with eps_d, the asymmetric model with the Hartree term in the state;
    sde_forms = 3 takes the mean of the three forms of the SDE.
    Returns (channels, Sigma, residuals), plus Sigma_H with eps_d."""
    n = grid.n
    outs = [alloc_channel(n) for _ in range(3)]
    dev = torch.device("cuda", torch.cuda.current_device())
    sigma = torch.zeros((n, 4), dtype=torch.complex128, device=dev)
    res = (C.c_double * max_iterations)()
    its = C.c_int(0)
    sH = C.c_double(0.0)
    D = (KqftChout * 3)(*[_chout(o, n) for o in outs])
    gc, qb, ql = grid.c(), q_bubble.c(), q_loop.c()
    aam = eps_d is not None
    if aam and q_hartree is None:
        raise ValueError("the asymmetric model needs q_hartree")
    qh = q_hartree.c() if aam else KqftQuad(1, QUAD_TAN_INFINITE, 0.0, 1.0)
    po = KqftParquetOpts(alpha, max_iterations, tol, depth, int(reduce_alpha), alpha_min, int(aam),
                         eps_d if aam else 0.0, qh, hartree_tol, sde_forms)
    _check(lib().kqft_parquet_solve(ctx(), C.byref(gc), C.c_double(U), C.c_double(Delta), C.c_double(T),
                                    C.byref(qb), C.byref(ql), C.byref(_opts(precision, KALL, 0, 0)), C.byref(po),
                                    D, C.c_void_p(sigma.data_ptr()), C.byref(sH), res, C.byref(its),
                                    _stream(stream)))
    out = (outs, sigma, [res[i] for i in range(its.value)])
    return out + (sH.value,) if aam else out


def bubble_adjoint(channel: int, left: Vertex, right: Vertex, G: Propagator, q: Quad, dout: Channel,
                   pi_kind: int = PI_GG, dleft: Optional[list] = None, dright: Optional[list] = None,
                   omega_batch: int = 0, stream=None, precision: int = FP64):
    """Accumulates cotangents into dleft[r] / dright[r] (Channels, or None to skip) and returns
    the device tensor dscal = (d left.r0, d right.r0, d G.Delta).  precision: FP64, or
    SPLIT_FP32 for the transposed products on FP32 MFMA."""
    n = left.grid.n
    dev = torch.device("cuda", torch.cuda.current_device())
    dscal = torch.zeros(3, dtype=torch.float64, device=dev)
    DL = (KqftChout * 3)(*[_chout_opt(d, n) for d in (dleft or [None] * 3)])
    DR = (KqftChout * 3)(*[_chout_opt(d, n) for d in (dright or [None] * 3)])
    lc, rc, gc, qc, oc = left.c(), right.c(), G.c(), q.c(), _chout(dout, n)
    _check(lib().kqft_bubble_adjoint(ctx(), channel, C.byref(lc), C.byref(rc), C.byref(gc), pi_kind, C.byref(qc),
                                     C.byref(_opts(precision, KALL, 1, omega_batch)), C.byref(oc), DL, DR,
                                     C.c_void_p(dscal.data_ptr()), _stream(stream)))
    return dscal


def sde_adjoint(gamma: Vertex, G: Propagator, q_bubble: Quad, q_loop: Quad, dsigma: torch.Tensor,
                dgamma: Optional[list] = None, stream=None):
    """Accumulates into dgamma[r] (Channels or None) and returns dscal = (d gamma.r0, d G.Delta)."""
    n = gamma.grid.n
    dev = torch.device("cuda", torch.cuda.current_device())
    dscal = torch.zeros(2, dtype=torch.float64, device=dev)
    empty = KqftChout(None, None, None, None)
    DG = (KqftChout * 3)(*[(_chout(d, n) if d is not None else empty) for d in (dgamma or [None] * 3)])
    vc, gc, qb, ql = gamma.c(), G.c(), q_bubble.c(), q_loop.c()
    ds = dsigma.contiguous()
    _ptr(ds, (n, 4), "dsigma")
    _check(lib().kqft_sde_adjoint(ctx(), C.byref(vc), C.byref(gc), C.byref(qb), C.byref(ql),
                                  C.byref(_opts(FP64, KALL, 0, 0)), C.c_void_p(ds.data_ptr()), DG,
                                  C.c_void_p(dscal.data_ptr()), _stream(stream)))
    return dscal


def mloop_adjoint(gamma: Vertex, G: Propagator, q: Quad, nloops: int, dgdot: Sequence[Sequence[Optional[Channel]]],
                  dgamma: Optional[list] = None, stream=None, precision: int = FP64):
    """Vector-Jacobian product of mloop_step for one point: dgdot[l][r] is the cotangent of
    the order-(l+1) insertion of channel r (a Channel, None = zero; a class left None counts as
    zero).  Accumulates into dgamma[r] (Channels, or None to skip) and returns the device
    tensor dscal = (d gamma.r0, d G.Delta)."""
    n = gamma.grid.n
    dev = torch.device("cuda", torch.cuda.current_device())
    dscal = torch.zeros(2, dtype=torch.float64, device=dev)
    empty = KqftChout(None, None, None, None)

    def co(c):
        if c is None:
            return empty
        return KqftChout(*[_ptr(getattr(c, x), class_shape(x, n), x) if getattr(c, x) is not None else None
                           for x in CLASSES])

    D = (KqftChout * (nloops * 3))(*[co(dgdot[l][r]) for l in range(nloops) for r in range(3)])
    DG = (KqftChout * 3)(*[_chout_opt(d, n) for d in (dgamma or [None] * 3)])
    vc, gc, qc = gamma.c(), G.c(), q.c()
    _check(lib().kqft_mloop_adjoint(ctx(), C.byref(vc), C.byref(gc), C.byref(qc), nloops,
                                    C.byref(_opts(precision, KALL, 0, 0)), D, DG, C.c_void_p(dscal.data_ptr()),
                                    _stream(stream)))
    return dscal


def mloop_jvp(gamma: Vertex, tangent: Vertex, G: Propagator, q: Quad, nloops: int, precision: int = FP64,
              omega_batch: int = 0, stream=None):
    """Insertions of mloop_step for one point and their tangents along the vertex tangent
    (fixed propagator): (out, dout), each out[l][r] a Channel."""
    n = gamma.grid.n
    outs = [[alloc_channel(n) for _ in range(3)] for _ in range(nloops)]
    douts = [[alloc_channel(n) for _ in range(3)] for _ in range(nloops)]
    O_ = (KqftChout * (nloops * 3))(*[_chout(outs[l][r], n) for l in range(nloops) for r in range(3)])
    D_ = (KqftChout * (nloops * 3))(*[_chout(douts[l][r], n) for l in range(nloops) for r in range(3)])
    vc, tc, gc, qc = gamma.c(), tangent.c(), G.c(), q.c()
    _check(lib().kqft_mloop_jvp(ctx(), C.byref(vc), C.byref(tc), C.byref(gc), C.byref(qc), nloops,
                                C.byref(_opts(precision, KALL, 0, omega_batch)), O_, D_, _stream(stream)))
    return outs, douts


def chi_noalloc(channel: int, gamma: Vertex, G: Propagator, q: Quad, out: torch.Tensor, stream=None) -> torch.Tensor:
    """kqft_chi without device allocations: writes chi_r into the caller's out [2, n, 16]
    complex128 (the library's static scratch holds every intermediate)."""
    n = gamma.grid.n
    _ptr(out, (2, n, 16), "out")
    vc, gc, qc = gamma.c(), G.c(), q.c()
    _check(lib().kqft_chi_noalloc(channel, C.byref(vc), C.byref(gc), C.byref(qc), C.c_void_p(out.data_ptr()),
                                  _stream(stream)))
    return out


def workspace_bytes():
    """(current, peak) device bytes of the library's workspaces."""
    cur, pk = C.c_size_t(), C.c_size_t()
    _check(lib().kqft_workspace_bytes(C.byref(cur), C.byref(pk)))
    return cur.value, pk.value


def workspace_reset_peak() -> None:
    """Restart the workspace peak at the current bytes (kqft_workspace_reset_peak)."""
    _check(lib().kqft_workspace_reset_peak())


def bubble_tune(channel: int, left: Vertex, right: Vertex, G: Propagator, q: Quad, pi_kind: int = PI_GG,
                precision: int = FP64, max_workspace: int = 0, out: Optional[Channel] = None, stream=None):
    """Autotune the transfer-frequency batch of this bubble shape (kqft_bubble_tune); the
    context keeps the winner for every later call with omega_batch = 0.  Returns (batch, ms)."""
    n = left.grid.n
    if out is None:
        out = alloc_channel(n)
    nb, ms = C.c_int(), C.c_double()
    lc, rc, gc, qc, oc = left.c(), right.c(), G.c(), q.c(), _chout(out, n)
    _check(lib().kqft_bubble_tune(ctx(), channel, C.byref(lc), C.byref(rc), C.byref(gc), pi_kind, C.byref(qc),
                                  C.byref(_opts(precision, KALL, 0, 0)), C.byref(oc), max_workspace, C.byref(nb),
                                  C.byref(ms), _stream(stream)))
    return nb.value, ms.value
