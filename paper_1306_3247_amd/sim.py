"""Thin ctypes binding of libwavepacket (include/wavepacket.h).

Argument marshalling only: every step of the propagation runs in the HIP
kernels of the library.  PyTorch provides the device memory of the state and
the stream the library enqueues on.  If the compiled library is missing the
import fails: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwavepacket.so")

WP_C64, WP_C128, WP_C64X = 1, 2, 3
PRECISIONS = {"c64": WP_C64, "c128": WP_C128, "c64x": WP_C64X}
WAVE_KINDS = {"const": 0, "sin": 1, "cos": 2, "gauss_cos": 3, "sin2_cos": 4}
V0_KINDS = {"none": 0, "softcore": 1, "morse": 2}
ORDERS = {"vkv": 0, "kvk": 1}
STATUS = {0: "WP_OK", -1: "WP_EINVAL", -2: "WP_ENOMEM", -3: "WP_EDEVICE",
          -4: "WP_EUNSUPPORTED", -5: "WP_ESTATE"}
OBSERVABLES = ("norm", "x", "y", "z", "x2", "y2", "z2", "energy", "sx", "sy", "sz", "autocorrelation")
OBS_ALL = 0xFF
OBS_ALL_EXT = 0xFFF
OBS_NORM = 0x1
OBS_MOMENTS = 0x7E | 0x700  # <x_d>, <x_d^2> and the widths


class WavepacketError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}" + (f" ({detail})" if detail else ""))


class Waveform(C.Structure):
    _fields_ = [("kind", C.c_int32), ("A0", C.c_double), ("A1", C.c_double),
                ("omega", C.c_double), ("phase", C.c_double), ("tc", C.c_double),
                ("tau", C.c_double), ("ti", C.c_double), ("tf", C.c_double)]


class GridDesc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("prec", C.c_int32), ("n", C.c_uint64 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("mass", C.c_double),
                ("hbar", C.c_double), ("dt", C.c_double)]


class PotentialDesc(C.Structure):
    _fields_ = [("a", Waveform * 3), ("b", Waveform * 3), ("c", Waveform), ("s", Waveform),
                ("v0_kind", C.c_int32), ("v0_par", C.c_double * 4)]


def _hip_runtimes() -> list:
    try:
        with open("/proc/self/maps") as f:
            return sorted({l.split()[-1] for l in f if "libamdhip64" in l and "r-xp" in l})
    except OSError:
        return []


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    # torch ships its own HIP runtime with the same soname as the system one.
    # Loading torch first makes the dynamic loader resolve the library's HIP
    # dependency to that same runtime, so torch's streams and allocations are
    # valid handles for the library.  Two runtimes in one process would not
    # share them.
    import torch  # noqa: F401

    L = C.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes are mapped in this process: {rts}")
    P, vp, u64, d = C.POINTER, C.c_void_p, C.c_uint64, C.c_double
    sig = {
        "wp_state_bytes": [P(GridDesc), P(u64)],
        "wp_state_pitch": [P(GridDesc), P(u64)],
        "wp_workspace_bytes": [P(GridDesc), P(u64)],
        "wp_create": [P(GridDesc), P(PotentialDesc), vp, P(vp)],
        "wp_destroy": [vp],
        "wp_bind_state": [vp, vp, u64],
        "wp_set_state": [vp, vp, d],
        "wp_set_state_gaussian": [vp, P(d), P(d), P(d), d],
        "wp_propagate": [vp, u64],
        "wp_set_order": [vp, C.c_int32],
        "wp_get_state": [vp, vp, C.c_int32],
        "wp_observables": [vp, C.c_uint32, P(d)],
        "wp_propagate_observe": [vp, u64, C.c_uint32, P(d)],
        "wp_propagate_observe_noalloc": [vp, u64, C.c_uint32, P(d)],
        "wp_get_time": [vp, P(d), P(u64)],
        "wp_synchronize": [vp],
        "wp_profile_propagate": [vp, u64, C.c_uint32, P(d), P(u64)],
        "wp_store_reference": [vp],
        "wp_time_pass": [vp, C.c_int32, C.c_uint32, P(d)],
        "wp_autotune": [vp, C.c_uint32, P(d)],
        "wp_set_slabs": [vp, C.c_uint32],
        "wp_batch_autotune": [vp, C.c_uint32],
        "wp_tune_get": [C.c_int32] * 5 + [P(C.c_int32)],
        "wp_tune_set": [C.c_int32] * 6,
        "wp_inner": [vp, vp, C.c_int32, P(d)],
        "wp_batch_create": [P(vp), C.c_uint32, vp, P(vp)],
        "wp_batch_set_graph_steps": [vp, C.c_uint32],
        "wp_batch_propagate": [vp, u64],
        "wp_batch_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.wp_state_ptr.argtypes = [vp]
    L.wp_state_ptr.restype = vp
    L.wp_last_error.argtypes = [vp]
    L.wp_last_error.restype = C.c_char_p
    L.wp_version.restype = C.c_char_p
    L.wp_batch_last_error.argtypes = [vp]
    L.wp_batch_last_error.restype = C.c_char_p
    L.wp_tune_clear.argtypes = []
    L.wp_tune_clear.restype = None
    L.wp_get_slabs.argtypes = [vp]
    L.wp_get_slabs.restype = C.c_uint32
    return L


lib = _load()


def _wave(w) -> Waveform:
    s = Waveform()
    if w is None:
        return s
    s.kind = WAVE_KINDS[w.kind] if isinstance(w.kind, str) else int(w.kind)
    for f in ("A0", "A1", "omega", "phase", "tc", "tau", "ti", "tf"):
        setattr(s, f, float(getattr(w, f)))
    return s


def grid_desc(grid, precision: str) -> GridDesc:
    g = GridDesc()
    g.ndim = int(grid.ndim)
    g.prec = PRECISIONS[precision]
    n = list(grid.n) + [1] * (3 - len(grid.n))
    lo = list(grid.lo) + [0.0] * (3 - len(grid.lo))
    hi = list(grid.hi) + [1.0] * (3 - len(grid.hi))
    for k in range(3):
        g.n[k], g.lo[k], g.hi[k] = int(n[k]), float(lo[k]), float(hi[k])
    g.mass, g.hbar, g.dt = float(grid.mass), float(grid.hbar), float(grid.dt)
    return g


def potential_desc(pot) -> PotentialDesc:
    p = PotentialDesc()
    for k in range(3):
        p.a[k] = _wave(pot.a[k] if k < len(pot.a) else None)
        p.b[k] = _wave(pot.b[k] if k < len(pot.b) else None)
    p.c, p.s = _wave(pot.c), _wave(pot.s)
    p.v0_kind = V0_KINDS[pot.v0_kind] if isinstance(pot.v0_kind, str) else int(pot.v0_kind)
    par = list(pot.v0_par) + [0.0] * (4 - len(pot.v0_par))
    for k in range(4):
        p.v0_par[k] = float(par[k])
    return p


def state_bytes(grid, precision: str) -> int:
    out = C.c_uint64()
    rc = lib.wp_state_bytes(C.byref(grid_desc(grid, precision)), C.byref(out))
    if rc:
        raise WavepacketError(rc, "wp_state_bytes")
    return out.value


def state_pitch(grid, precision: str) -> int:
    """Points between the first-axis planes of the state in device memory."""
    out = C.c_uint64()
    rc = lib.wp_state_pitch(C.byref(grid_desc(grid, precision)), C.byref(out))
    if rc:
        raise WavepacketError(rc, "wp_state_pitch")
    return out.value


def workspace_bytes(grid, precision: str) -> int:
    out = C.c_uint64()
    rc = lib.wp_workspace_bytes(C.byref(grid_desc(grid, precision)), C.byref(out))
    if rc:
        raise WavepacketError(rc, "wp_workspace_bytes")
    return out.value


PASS_KIND_IDS = {"fft": 0, "potential": 1, "kinetic": 2, "split_potential": 3, "split_kinetic": 4}
TUNE_VARIANTS = 4
TUNE_SLAB_CHOICES = 8


def tune_get(batched: bool, precision: str, lg_n: int, strided: bool, kind: str) -> int:
    """Variant in the process-wide tuning table for one pass shape."""
    out = C.c_int32()
    rc = lib.wp_tune_get(int(batched), PRECISIONS[precision], int(lg_n), int(strided), PASS_KIND_IDS[kind],
                         C.byref(out))
    if rc:
        raise WavepacketError(rc, "wp_tune_get")
    return out.value


def tune_set(batched: bool, precision: str, lg_n: int, strided: bool, kind: str, variant: int) -> None:
    rc = lib.wp_tune_set(int(batched), PRECISIONS[precision], int(lg_n), int(strided), PASS_KIND_IDS[kind],
                         int(variant))
    if rc:
        raise WavepacketError(rc, "wp_tune_set")


def tune_clear() -> None:
    lib.wp_tune_clear()


def _arr3(v, fill: float):
    a = (C.c_double * 3)()
    vals = list(v) + [fill] * (3 - len(v))
    for k in range(3):
        a[k] = float(vals[k])
    return a


class Simulation:
    """One solver handle.  The state lives in a torch-allocated device buffer
    bound to the handle; work is ordered on `stream` (a torch.cuda.Stream,
    default: torch's current stream)."""

    def __init__(self, grid, pot, precision: str = "c128", stream=None, order: str = "vkv"):
        import torch  # device memory and streams only

        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.grid, self.precision = grid, precision
        self.shape = tuple((list(grid.n) + [1, 1, 1])[: int(grid.ndim)])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._g = grid_desc(grid, precision)
        self._p = potential_desc(pot)
        h = C.c_void_p()
        rc = lib.wp_create(C.byref(self._g), C.byref(self._p), C.c_void_p(self.stream.cuda_stream),
                           C.byref(h))
        if rc:
            raise WavepacketError(rc, "wp_create")
        self._h = h
        nbytes = state_bytes(grid, precision)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._check(lib.wp_bind_state(self._h, C.c_void_p(self.buffer.data_ptr()), nbytes), "wp_bind_state")
        if order != "vkv":
            self.set_order(order)

    def _check(self, rc: int, what: str) -> None:
        if rc:
            raise WavepacketError(rc, what, lib.wp_last_error(self._h).decode())

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.wp_destroy(self._h)
            self._h = None
            self.buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_order(self, order: str) -> None:
        self._check(lib.wp_set_order(self._h, ORDERS[order]), "wp_set_order")

    def set_state(self, psi: np.ndarray, t0: float = 0.0) -> None:
        a = np.ascontiguousarray(psi, dtype=np.complex128)
        if a.size != int(np.prod(self.shape)):
            raise ValueError("state size does not match the grid")
        self._check(lib.wp_set_state(self._h, C.c_void_p(a.ctypes.data), float(t0)), "wp_set_state")

    def set_gaussian(self, center, sigma, k, t0: float = 0.0) -> None:
        self._check(lib.wp_set_state_gaussian(self._h, _arr3(center, 0.0), _arr3(sigma, 1.0),
                                              _arr3(k, 0.0), float(t0)), "wp_set_state_gaussian")

    def propagate(self, nsteps: int) -> None:
        self._check(lib.wp_propagate(self._h, int(nsteps)), "wp_propagate")

    def get_state(self, as_precision: str = "c128") -> np.ndarray:
        dt = np.complex128 if as_precision == "c128" else np.complex64
        out = np.empty(self.shape, dtype=dt)
        self._check(lib.wp_get_state(self._h, C.c_void_p(out.ctypes.data), PRECISIONS[as_precision]),
                    "wp_get_state")
        return out

    def observables(self, mask: int = OBS_ALL) -> dict:
        out = (C.c_double * 12)()
        self._check(lib.wp_observables(self._h, int(mask), out), "wp_observables")
        return {k: out[i] for i, k in enumerate(OBSERVABLES) if mask & (1 << i)}

    def propagate_observe(self, nsteps: int, mask: int = OBS_NORM | OBS_MOMENTS) -> dict:
        """Propagate nsteps steps and return the observables of the final
        state (see wp_propagate_observe: moments come from the pass that
        ends the propagation where the grid allows)."""
        out = (C.c_double * 12)()
        self._check(lib.wp_propagate_observe(self._h, int(nsteps), int(mask), out), "wp_propagate_observe")
        return {k: out[i] for i, k in enumerate(OBSERVABLES) if mask & (1 << i)}

    def propagate_observe_noalloc(self, nsteps: int, mask: int = OBS_NORM | OBS_MOMENTS) -> dict:
        """As propagate_observe, allocating nothing (see
        wp_propagate_observe_noalloc: the fused moments only, with the moment
        rows in the library's fixed per-device array)."""
        out = (C.c_double * 12)()
        self._check(lib.wp_propagate_observe_noalloc(self._h, int(nsteps), int(mask), out),
                    "wp_propagate_observe_noalloc")
        return {k: out[i] for i, k in enumerate(OBSERVABLES) if mask & (1 << i)}

    def store_reference(self) -> None:
        """Keep the current state as the reference of the autocorrelation."""
        self._check(lib.wp_store_reference(self._h), "wp_store_reference")

    def inner(self, phi) -> complex:
        """<phi|psi> over the grid; phi is a device tensor (complex64 or
        complex128, the state's shape) or a host array (copied to the device)."""
        import torch

        if isinstance(phi, np.ndarray):
            phi = torch.from_numpy(np.ascontiguousarray(phi)).to("cuda")
        if phi.dtype not in (torch.complex64, torch.complex128) or not phi.is_cuda:
            raise ValueError("phi must be a complex64/complex128 CUDA tensor or a numpy array")
        if phi.numel() != int(np.prod(self.shape)) or not phi.is_contiguous():
            raise ValueError("phi must be contiguous with the state's size")
        prec = WP_C128 if phi.dtype == torch.complex128 else WP_C64
        # the copy above ran on torch's current stream; order the read after it
        self.stream.wait_stream(torch.cuda.current_stream())
        out = (C.c_double * 2)()
        self._check(lib.wp_inner(self._h, C.c_void_p(phi.data_ptr()), prec, out), "wp_inner")
        return complex(out[0], out[1])

    def time(self):
        t, n = C.c_double(), C.c_uint64()
        self._check(lib.wp_get_time(self._h, C.byref(t), C.byref(n)), "wp_get_time")
        return t.value, n.value

    def synchronize(self) -> None:
        self._check(lib.wp_synchronize(self._h), "wp_synchronize")

    PASS_KINDS = ("solve1d", "axis0", "mid_fwd", "last", "mid_inv", "edge", "coef")

    def profile_propagate(self, nsteps: int, kinds=None) -> dict:
        """Propagate with an event pair attached to the dispatch of every
        kernel of the given classes (names from PASS_KINDS; all by default);
        returns {kind: (launches, total_ms)} for the timed kinds that ran."""
        mask = 0xFFFFFFFF if kinds is None else sum(1 << self.PASS_KINDS.index(k) for k in kinds)
        ms = (C.c_double * 8)()
        cnt = (C.c_uint64 * 8)()
        self._check(lib.wp_profile_propagate(self._h, int(nsteps), mask, ms, cnt), "wp_profile_propagate")
        return {k: (cnt[i], ms[i]) for i, k in enumerate(self.PASS_KINDS) if cnt[i]}

    def time_pass(self, kind: str, reps: int = 20) -> float:
        """Average device milliseconds of one line pass of class `kind`
        (see PASS_KINDS) over `reps` back-to-back launches.  Measurement
        only: the state is not a solution afterwards."""
        ms = C.c_double()
        self._check(lib.wp_time_pass(self._h, self.PASS_KINDS.index(kind), int(reps), C.byref(ms)), "wp_time_pass")
        return ms.value

    TUNE_CLASSES = ("axis0", "mid", "last")

    def autotune(self, reps: int = 10) -> dict:
        """Tune this grid's line passes (see wp_autotune): the fastest
        variant of each class goes to the tuning table and the fastest slab
        count to this handle.  Returns {class: {variant: ms per step}} and
        "slabs": {count: ms per step} for what was timed."""
        ms = (C.c_double * (3 * TUNE_VARIANTS + TUNE_SLAB_CHOICES))()
        self._check(lib.wp_autotune(self._h, int(reps), ms), "wp_autotune")
        out = {}
        for c, name in enumerate(self.TUNE_CLASSES):
            row = {v: ms[c * TUNE_VARIANTS + v] for v in range(TUNE_VARIANTS)
                   if ms[c * TUNE_VARIANTS + v] == ms[c * TUNE_VARIANTS + v]}
            if row:
                out[name] = row
        slabs = {1 << k: ms[3 * TUNE_VARIANTS + k] for k in range(TUNE_SLAB_CHOICES)
                 if ms[3 * TUNE_VARIANTS + k] == ms[3 * TUNE_VARIANTS + k]}
        if slabs:
            out["slabs"] = slabs
        return out

    def set_slabs(self, count: int) -> None:
        """x slabs of the middle passes of a 3D step (see wp_set_slabs)."""
        self._check(lib.wp_set_slabs(self._h, int(count)), "wp_set_slabs")

    def slabs(self) -> int:
        return int(lib.wp_get_slabs(self._h))

    def state_ptr(self) -> int:
        return lib.wp_state_ptr(self._h)

    def state_tensor(self):
        """The state in device memory as a complex tensor of the grid's shape
        (a strided view of the bound buffer, no copy): complex128 for the
        FP64 state, complex64 otherwise."""
        import torch

        dt = torch.complex128 if self.precision == "c128" else torch.complex64
        flat = self.buffer.view(dt)
        n0 = self.shape[0]
        plane = int(np.prod(self.shape[1:])) if len(self.shape) > 1 else 1
        pitch = state_pitch(self.grid, self.precision)
        strides = [pitch] + [int(np.prod(self.shape[d + 1:])) for d in range(1, len(self.shape))]
        assert flat.numel() >= (n0 - 1) * pitch + plane
        return flat.as_strided(self.shape, strides)


def from_problem(prob, precision: Optional[str] = None, stream=None, order: str = "vkv") -> Simulation:
    """Create a Simulation for a workloads.Problem and set its Gaussian state."""
    s = Simulation(prob.grid, prob.pot, precision or prob.precision, stream=stream, order=order)
    s.set_gaussian(prob.init.center, prob.init.sigma, prob.init.k, prob.t0)
    return s


class Batch:
    """Several Simulations advanced together with shared launches (see
    wp_batch_create).  The members stay usable for get_state/observables;
    advance them through the batch while it exists."""

    def __init__(self, sims, stream=None, graph_steps: int = 0):
        import torch

        if not sims:
            raise ValueError("empty batch")
        self.sims = list(sims)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (C.c_void_p * len(self.sims))(*[s._h.value for s in self.sims])
        h = C.c_void_p()
        rc = lib.wp_batch_create(arr, len(self.sims), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise WavepacketError(rc, "wp_batch_create")
        self._h = h
        if graph_steps:
            self._check(lib.wp_batch_set_graph_steps(self._h, int(graph_steps)), "wp_batch_set_graph_steps")

    def _check(self, rc: int, what: str) -> None:
        if rc:
            raise WavepacketError(rc, what, lib.wp_batch_last_error(self._h).decode())

    def propagate(self, nsteps: int) -> None:
        self._check(lib.wp_batch_propagate(self._h, int(nsteps)), "wp_batch_propagate")

    def autotune(self, reps: int = 10) -> None:
        """Pick the fastest kernel variant of each pass group (members'
        states are saved and restored)."""
        self._check(lib.wp_batch_autotune(self._h, int(reps)), "wp_batch_autotune")

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.wp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
