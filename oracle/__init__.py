"""Plain FP64 CPU oracle of the split-operator time step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports,
links or runs anything in this folder, and this folder never imports the GPU
package.  Problem descriptions are read by attribute (duck typing), so the
seeded input generators can feed both sides without either importing the other.

Functions follow the paper (Dion, Hashemloo, Rahali, Comput. Phys. Commun.):
grid of Section 2.1 (eqs. grid, Deltax), momentum grid after eq. ft, step of
eq. splitop in the V-K-V order with trapezoid time sampling (or the printed
K-V-K midpoint order), observables of Table 3 and the utilities of Section 3.2.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

WAVE_KINDS = {"const": 0, "sin": 1, "cos": 2, "gauss_cos": 3, "sin2_cos": 4}
V0_KINDS = {"none": 0, "softcore": 1, "morse": 2}
ORDER_VKV, ORDER_KVK = 0, 1


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fused multiply-add)."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fcx-limited-range", "-Wall", "-o", LIB_PATH + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Wave(C.Structure):
    _fields_ = [("kind", C.c_int32), ("A0", C.c_double), ("A1", C.c_double),
                ("omega", C.c_double), ("phase", C.c_double), ("tc", C.c_double),
                ("tau", C.c_double), ("ti", C.c_double), ("tf", C.c_double)]


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int64 * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("mass", C.c_double), ("hbar", C.c_double),
                ("dt", C.c_double)]


class _Pot(C.Structure):
    _fields_ = [("a", _Wave * 3), ("b", _Wave * 3), ("c", _Wave), ("s", _Wave),
                ("v0_kind", C.c_int32), ("v0_par", C.c_double * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        d = C.c_double
        L.orc_wave_eval.restype = d
        L.orc_wave_eval.argtypes = [P(_Wave), d]
        for name in ("orc_coords", "orc_wavenumbers"):
            getattr(L, name).argtypes = [P(_Grid), C.c_int, C.c_void_p]
        L.orc_potential.argtypes = [P(_Grid), P(_Pot), d, C.c_void_p]
        L.orc_dft1d.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int]
        L.orc_fft1d.argtypes = [C.c_int64, C.c_void_p, C.c_int]
        L.orc_fftn.argtypes = [P(_Grid), C.c_void_p, C.c_int]
        L.orc_gaussian.argtypes = [P(_Grid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_propagate.argtypes = [P(_Grid), P(_Pot), C.c_void_p, d, C.c_int64, C.c_int64, C.c_int]
        L.orc_observables.argtypes = [P(_Grid), P(_Pot), C.c_void_p, d, C.c_void_p]
        L.orc_inner.argtypes = [P(_Grid), C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# --- descriptor conversion (attribute access only) ---------------------------

def _grid(g) -> _Grid:
    s = _Grid()
    s.ndim = int(g.ndim)
    n = list(g.n) + [1] * (3 - len(g.n))
    lo = list(g.lo) + [0.0] * (3 - len(g.lo))
    hi = list(g.hi) + [1.0] * (3 - len(g.hi))
    for d in range(3):
        s.n[d] = int(n[d])
        s.lo[d] = float(lo[d])
        s.hi[d] = float(hi[d])
    s.mass, s.hbar, s.dt = float(g.mass), float(g.hbar), float(g.dt)
    return s


def _wave(w) -> _Wave:
    s = _Wave()
    if w is None:
        s.kind = 0
        return s
    s.kind = WAVE_KINDS[w.kind] if isinstance(w.kind, str) else int(w.kind)
    for f in ("A0", "A1", "omega", "phase", "tc", "tau", "ti", "tf"):
        setattr(s, f, float(getattr(w, f, 0.0)))
    return s


def _pot(p) -> _Pot:
    s = _Pot()
    for d in range(3):
        s.a[d] = _wave(p.a[d] if d < len(p.a) else None)
        s.b[d] = _wave(p.b[d] if d < len(p.b) else None)
    s.c = _wave(p.c)
    s.s = _wave(p.s)
    s.v0_kind = V0_KINDS[p.v0_kind] if isinstance(p.v0_kind, str) else int(p.v0_kind)
    par = list(p.v0_par) + [0.0] * (4 - len(p.v0_par))
    for i in range(4):
        s.v0_par[i] = float(par[i])
    return s


def shape(g) -> tuple:
    n = list(g.n) + [1] * (3 - len(g.n))
    return tuple(int(v) for v in n[: int(g.ndim)])


def _state(g, psi) -> np.ndarray:
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    if a.size != int(np.prod(shape(g))):
        raise ValueError("state size does not match the grid")
    return a


# --- public functions ---------------------------------------------------------

def num_threads() -> int:
    return lib().orc_num_threads()


def wave_eval(w, t: float) -> float:
    s = _wave(w)
    return lib().orc_wave_eval(C.byref(s), float(t))


def coords(g, axis: int) -> np.ndarray:
    gs = _grid(g)
    out = np.empty(gs.n[axis], dtype=np.float64)
    _check(lib().orc_coords(C.byref(gs), axis, _ptr(out)), "coords")
    return out


def wavenumbers(g, axis: int) -> np.ndarray:
    gs = _grid(g)
    out = np.empty(gs.n[axis], dtype=np.float64)
    _check(lib().orc_wavenumbers(C.byref(gs), axis, _ptr(out)), "wavenumbers")
    return out


def potential(g, p, t: float) -> np.ndarray:
    gs, ps = _grid(g), _pot(p)
    out = np.empty(shape(g), dtype=np.float64)
    _check(lib().orc_potential(C.byref(gs), C.byref(ps), float(t), _ptr(out)), "potential")
    return out


def dft(x, direction: int = -1) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.complex128).ravel()
    out = np.empty_like(a)
    _check(lib().orc_dft1d(a.size, _ptr(a), _ptr(out), int(direction)), "dft")
    return out


def fft(x, direction: int = -1) -> np.ndarray:
    a = np.array(x, dtype=np.complex128).ravel()
    _check(lib().orc_fft1d(a.size, _ptr(a), int(direction)), "fft")
    return a


def fftn(g, psi, direction: int = -1) -> np.ndarray:
    gs = _grid(g)
    a = _state(g, psi).copy()
    _check(lib().orc_fftn(C.byref(gs), _ptr(a), int(direction)), "fftn")
    return a


def gaussian(g, center, sigma, k) -> np.ndarray:
    gs = _grid(g)
    pad = lambda v, f: np.array(list(v) + [f] * (3 - len(v)), dtype=np.float64)
    c, s, kk = pad(center, 0.0), pad(sigma, 1.0), pad(k, 0.0)
    out = np.empty(shape(g), dtype=np.complex128)
    _check(lib().orc_gaussian(C.byref(gs), _ptr(c), _ptr(s), _ptr(kk), _ptr(out)), "gaussian")
    return out


def propagate(g, p, psi, nsteps: int, t0: float = 0.0, n0: int = 0,
              order: int = ORDER_VKV) -> np.ndarray:
    """Return psi after nsteps steps; step n starts at t0 + n*dt, n = n0, n0+1, ..."""
    gs, ps = _grid(g), _pot(p)
    a = _state(g, psi).copy()
    _check(lib().orc_propagate(C.byref(gs), C.byref(ps), _ptr(a), float(t0), int(n0),
                               int(nsteps), int(order)), "propagate")
    return a


OBSERVABLES = ("norm", "x", "y", "z", "x2", "y2", "z2", "energy")


def observables(g, p, psi, t: float) -> dict:
    gs, ps = _grid(g), _pot(p)
    a = _state(g, psi)
    out = np.zeros(8, dtype=np.float64)
    _check(lib().orc_observables(C.byref(gs), C.byref(ps), _ptr(a), float(t), _ptr(out)),
           "observables")
    return dict(zip(OBSERVABLES, out.tolist()))


def inner(g, f1, f2) -> complex:
    gs = _grid(g)
    a, b = _state(g, f1), _state(g, f2)
    out = np.zeros(2, dtype=np.float64)
    _check(lib().orc_inner(C.byref(gs), _ptr(a), _ptr(b), _ptr(out)), "inner")
    return complex(out[0], out[1])
