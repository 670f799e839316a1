"""Problem descriptions and seeded synthetic inputs.

This module holds parameter containers and seeded random draws only: no step
of the method is computed here.  The test suite and the benchmark hand the same
descriptions to the GPU library and to the CPU oracle; neither of those imports
the other.

Workloads (synthetic; the paper measures no public dataset):
  * driven harmonic oscillator, 1D, 1024 points;
  * modulated 2D trap, 1024 x 1024;
  * soft-core 3D atom in a Gaussian-envelope pulse, 512^3 (the throughput
    workload);
  * a batch of 256 independent 2D driven traps with seeded sizes and drives;
  * a Poisson stream of mixed 1D/2D/3D requests (serving);
  * the Ba+ ion in a Paul trap of Section 4.2, 512^3 in SI units.
The Gaussian initial state follows Section 4.2 of the paper.
"""
from __future__ import annotations

import dataclasses as dc
from typing import List, Optional, Sequence

import numpy as np


@dc.dataclass
class Wave:
    """f(t) = A0 + A1 * env(t) * trig(omega t + phase); see the `kind` list."""
    kind: str = "const"  # const | sin | cos | gauss_cos | sin2_cos
    A0: float = 0.0
    A1: float = 0.0
    omega: float = 0.0
    phase: float = 0.0
    tc: float = 0.0
    tau: float = 1.0
    ti: float = 0.0
    tf: float = 1.0


def const(v: float) -> Wave:
    return Wave("const", A0=v)


@dc.dataclass
class Grid:
    ndim: int
    n: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    mass: float = 1.0
    hbar: float = 1.0
    dt: float = 0.01

    def full_n(self) -> List[int]:
        return [int(v) for v in self.n] + [1] * (3 - len(self.n))

    def shape(self) -> tuple:
        return tuple(self.full_n()[: self.ndim])

    def points(self) -> int:
        return int(np.prod(self.full_n()))


@dc.dataclass
class Potential:
    """V(x,t) = c(t) + sum_d [a_d(t) x_d + b_d(t) x_d^2] + s(t) V0(x)."""
    a: List[Wave] = dc.field(default_factory=lambda: [Wave(), Wave(), Wave()])
    b: List[Wave] = dc.field(default_factory=lambda: [Wave(), Wave(), Wave()])
    c: Wave = dc.field(default_factory=Wave)
    s: Wave = dc.field(default_factory=Wave)
    v0_kind: str = "none"  # none | softcore | morse
    v0_par: Sequence[float] = (0.0, 0.0, 0.0, 0.0)


@dc.dataclass
class Gaussian:
    center: Sequence[float]
    sigma: Sequence[float]
    k: Sequence[float]


@dc.dataclass
class Problem:
    name: str
    grid: Grid
    pot: Potential
    init: Gaussian
    steps: int
    precision: str = "c128"  # c128 | c64
    t0: float = 0.0


# --- named workloads ----------------------------------------------------------

def driven_ho_1d(n: int = 1024, steps: int = 1000, precision: str = "c128") -> Problem:
    """1D, hbar = m = 1, [-20, 20), V = x^2/2 - E0 x sin(omega t), E0 = 0.1,
    omega = 1; Gaussian at -5, sigma 1, k 2; dt 0.01."""
    g = Grid(1, [n], [-20.0], [20.0], dt=0.01)
    p = Potential()
    p.b[0] = const(0.5)
    p.a[0] = Wave("sin", A0=0.0, A1=-0.1, omega=1.0)
    return Problem("driven_ho_1d", g, p, Gaussian([-5.0], [1.0], [2.0]), steps, precision)


def modulated_trap_2d(n: int = 1024, steps: int = 2000, precision: str = "c128",
                      half_width: float = 32.0) -> Problem:
    """2D on [-32, 32)^2, V = (1 + 0.3 cos 2t) x^2/2 + (1 - 0.3 cos 2t) y^2/2;
    Gaussian at (3, -2), sigma 1, k (0, 1); dt 0.005."""
    g = Grid(2, [n, n], [-half_width] * 2, [half_width] * 2, dt=0.005)
    p = Potential()
    p.b[0] = Wave("cos", A0=0.5, A1=0.15, omega=2.0)
    p.b[1] = Wave("cos", A0=0.5, A1=-0.15, omega=2.0)
    return Problem("modulated_trap_2d", g, p, Gaussian([3.0, -2.0], [1.0, 1.0], [0.0, 1.0]),
                   steps, precision)


def softcore_3d(n: int = 512, steps: int = 2000, precision: str = "c64",
                half_width: float = 40.0) -> Problem:
    """3D on [-40, 40)^3, V = -1/sqrt(r^2 + 1) + E(t) z,
    E(t) = 0.05 exp(-((t - 10)/4)^2) cos(1.5 t); Gaussian sigma 1 at the
    origin, k = 0; dt 0.01."""
    g = Grid(3, [n, n, n], [-half_width] * 3, [half_width] * 3, dt=0.01)
    p = Potential(v0_kind="softcore", v0_par=(1.0, 1.0, 0.0, 0.0))
    p.s = const(1.0)
    p.a[2] = Wave("gauss_cos", A0=0.0, A1=0.05, omega=1.5, tc=10.0, tau=4.0)
    return Problem("softcore_3d", g, p, Gaussian([0.0] * 3, [1.0] * 3, [0.0] * 3), steps, precision)


def driven_trap(ndim: int, n: int, E0: float, omega: float, center, k, steps: int,
                precision: str = "c64", half_width: float = 16.0, dt: float = 0.01) -> Problem:
    """V = |x|^2/2 - E0 x sin(omega t) on [-16, 16)^ndim (batch and serving)."""
    g = Grid(ndim, [n] * ndim, [-half_width] * ndim, [half_width] * ndim, dt=dt)
    p = Potential()
    for d in range(ndim):
        p.b[d] = const(0.5)
    p.a[0] = Wave("sin", A0=0.0, A1=-float(E0), omega=float(omega))
    return Problem(f"driven_trap_{ndim}d_{n}", g, p,
                   Gaussian(list(center), [1.0] * ndim, list(k)), steps, precision)


# CODATA 2010 values (the paper's constants reference) and the ion of
# Section 4.2.
HBAR_SI = 1.054571726e-34     # J s
E_CHARGE_SI = 1.602176565e-19  # C
BA138_MASS_SI = 2.28997005e-25  # kg


def paul_trap_3d(n: int = 512, steps: int = 18500, precision: str = "c64", half_width: float = 1e-6,
                 dt: float = 2e-9) -> Problem:
    """A 138Ba+ ion in a Paul trap (Section 4.2), SI units: V = Z e (U0 + V0
    cos(Omega t)) (x^2 + y^2 - 2 z^2) / (2 d^2) with Z = 1, U0 = 0, V0 = 200 V,
    Omega = 2 pi 18 MHz, d^2 = r0^2 + 2 z0^2, r0 = 1.6 mm, z0 = r0/sqrt(2);
    Gaussian at (2, 1, 2) x 1e-8 m with p = (1e-27, 0, 0) kg m/s and widths
    (7.342, 7.342, 5.192) x 1e-8 m; n^3 points on [-half_width, half_width)^3
    (the paper: 512 on [-1e-6, 1e-6) m), dt = 2 ns, 18500 steps."""
    U0, V0, Omega = 0.0, 200.0, 2.0 * np.pi * 18e6
    r0 = 1.6e-3
    z0 = r0 / np.sqrt(2.0)
    d2 = r0 * r0 + 2.0 * z0 * z0
    q = 1.0 * E_CHARGE_SI / (2.0 * d2)
    g = Grid(3, [n] * 3, [-half_width] * 3, [half_width] * 3, mass=BA138_MASS_SI, hbar=HBAR_SI, dt=dt)
    p = Potential()
    for d, f in ((0, 1.0), (1, 1.0), (2, -2.0)):
        p.b[d] = Wave("cos", A0=f * q * U0, A1=f * q * V0, omega=Omega)
    k = [1e-27 / HBAR_SI, 0.0, 0.0]
    init = Gaussian([2e-8, 1e-8, 2e-8], [7.342e-8, 7.342e-8, 5.192e-8], k)
    return Problem(f"paul_trap_3d_{n}", g, p, init, steps, precision)


def batch_2d(count: int = 256, seed: int = 1306, steps: int = 1000,
             sizes: Sequence[int] = (128, 256, 512), precision: str = "c64") -> List[Problem]:
    """Independent 2D driven traps: size uniform in `sizes`, E0 ~ U[0.01, 0.2],
    omega ~ U[0.5, 2], centre ~ U[-3, 3]^2, k ~ U[-1, 1]^2, sigma 1 (drawn in
    that order per solve from numpy's default_rng(seed))."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        E0 = float(rng.uniform(0.01, 0.2))
        omega = float(rng.uniform(0.5, 2.0))
        c = rng.uniform(-3.0, 3.0, size=2)
        k = rng.uniform(-1.0, 1.0, size=2)
        out.append(driven_trap(2, n, E0, omega, c, k, steps, precision))
    return out


@dc.dataclass
class Request:
    rid: int
    arrival: float  # seconds after the stream starts
    problem: Problem


def serving_stream(count: int, rate_hz: float, seed: int = 1306,
                   log2_1d: Sequence[int] = (10, 16), sizes_2d: Sequence[int] = (128, 256, 512, 1024),
                   sizes_3d: Sequence[int] = (64, 128, 256), steps_range=(500, 5000),
                   precision: str = "c64", fractions=(0.6, 0.3)) -> List[Request]:
    """Poisson arrivals at `rate_hz` (exponential gaps; rate_hz = inf puts
    every arrival at 0).  Mix: fractions[0] 1D with n = 2^k, k uniform in
    log2_1d (inclusive), on [-20, 20); fractions[1] 2D with n uniform in
    sizes_2d, on [-16, 16)^2; the rest 3D with n uniform in sizes_3d, on
    [-16, 16)^3.  Each is a driven trap V = |x|^2/2 - E0 x sin(omega t), E0 ~
    U[0.01, 0.2], omega ~ U[0.5, 2], Gaussian centre ~ U[-3, 3]^d, k ~
    U[-1, 1]^d, sigma 1, dt = 0.01, steps uniform in steps_range (inclusive),
    drawn per request in this order from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(count):
        if np.isfinite(rate_hz):
            t += float(rng.exponential(1.0 / rate_hz))
        u = float(rng.uniform())
        if u < fractions[0]:
            ndim, n = 1, 1 << int(rng.integers(log2_1d[0], log2_1d[1] + 1))
        elif u < fractions[0] + fractions[1]:
            ndim, n = 2, int(rng.choice(list(sizes_2d)))
        else:
            ndim, n = 3, int(rng.choice(list(sizes_3d)))
        E0 = float(rng.uniform(0.01, 0.2))
        omega = float(rng.uniform(0.5, 2.0))
        c = rng.uniform(-3.0, 3.0, size=ndim)
        k = rng.uniform(-1.0, 1.0, size=ndim)
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        half = 20.0 if ndim == 1 else 16.0
        reqs.append(Request(i, t, driven_trap(ndim, n, E0, omega, c, k, steps, precision, half)))
    return reqs


def random_state(shape, seed: int) -> np.ndarray:
    """Seeded complex normal test state (no normalisation)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
