"""Synthetic single-impurity Anderson model workloads (particle-hole symmetric,
flat hybridization, wide band).  Sizes follow the paper's workloads: a
non-uniform frequency grid dense near zero, 16 Keldysh x 2 spin components per
frequency point, three channels with four asymptotic classes each, and
resolutions from 31 to 201 points per frequency axis (the paper's largest
production run used 125).  The paper's benchmark data (NRG) are not available;
these seeded inputs stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

NOISE_AMPLITUDE = 1e-3
CLASSES = ("K1", "K2", "K2p", "K3")


@dataclass(frozen=True)
class Workload:
    name: str
    N: int                 # points per frequency axis (all classes share the grid)
    Nq: int                # Gauss-Legendre nodes of the bubble integral
    U: float = 1.0
    T: float = 0.1
    Delta: float = 1.0
    L: float = 20.0        # grid and quadrature extent [-L, L]
    a: float = 1.0         # tangent-map scale
    channels: tuple = ("a",)
    Nq_loop: Optional[int] = None  # loop (SDE) quadrature nodes, default = Nq


# The five workloads named in the build's target configuration, with readings
# for the parts the description leaves open (grid scale a = Delta, L = 20,
# T = 0.1 where unstated).
CONFIGS = {
    "bubble_a_n31": Workload("bubble_a_n31", 31, 201, U=1.0, T=0.1),
    "bubbles_sde_n101": Workload("bubbles_sde_n101", 101, 1001, U=1.0, T=0.05, channels=("a", "p", "t")),
    "bubble_a_n201": Workload("bubble_a_n201", 201, 2001, U=1.0, T=0.1),
    "adjoint_n151": Workload("adjoint_n151", 151, 1501, U=1.0, T=0.1),
}
THREE_CHANNEL_U_VALUES = (0.5, 1.0, 2.0)
# twelve uneven parameter points of the batched multiloop workload:
# U in {0.25, 0.5, 1, 1.5, 2, 3} (outer) x T in {0.01, 0.1}; N cycles through 51..201, Nq = 10N - 9
MULTILOOP_POINTS = [(U, T, [51, 101, 151, 201][i % 4]) for i, (U, T) in
             enumerate([(U, T) for U in (0.25, 0.5, 1.0, 1.5, 2.0, 3.0) for T in (0.01, 0.1)])]


def class_shape(name: str, N: int) -> tuple:
    return {"K1": (2, N, 16), "K2": (2, N, N, 16), "K2p": (2, N, N, 16), "K3": (2, N, N, N, 16)}[name]


def complex_noise(rng: np.random.Generator, shape: tuple, amplitude: float = NOISE_AMPLITUDE) -> np.ndarray:
    """amplitude * (z0 + i z1) with (z0, z1) consecutive standard normals, written straight
    into the interleaved (re, im) storage of the result."""
    out = np.empty(shape, dtype=np.complex128)
    view = out.view(np.float64).reshape(shape + (2,))
    rng.standard_normal(out=view)
    view *= amplitude
    return out


def seed_noise(N: int, seed: int = 0, amplitude: float = NOISE_AMPLITUDE, classes=CLASSES) -> list:
    """noise[r][cls] for r = a, p, t and cls in K1, K2, K2p, K3, drawn from one
    generator in that order (C order of [s][w][v][v'][16])."""
    rng = np.random.default_rng(seed)
    out = []
    for _r in range(3):
        d = {}
        for c in CLASSES:
            arr = complex_noise(rng, class_shape(c, N), amplitude)
            d[c] = arr if c in classes else None
        out.append(d)
    return out


def random_channel(N: int, seed: int, amplitude: float = 1.0) -> dict:
    """A generic random channel (all classes), for parity tests of arbitrary inputs."""
    rng = np.random.default_rng(seed)
    return {c: complex_noise(rng, class_shape(c, N), amplitude) for c in CLASSES}
