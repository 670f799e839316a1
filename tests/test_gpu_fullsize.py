"""GPU path at the full workload sizes, in the launch configuration bench.py
times.  Where the oracle cannot run the whole length, these check element-wise
parity for a few steps and properties that hold at any size for the rest:
norm, reversibility, the classical trajectory of <x> for quadratic
potentials, and the FP32 state against the (oracle-pinned) FP64 state after
the full step count."""
import math

import numpy as np
import pytest

from conftest import leapfrog, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


SOFTCORE_STEPS = 3


@pytest.fixture(scope="module")
def softcore_512_oracle(W, oracle_mod):
    """The oracle's 512^3 soft-core state after 3 steps from t0 = 9.5 (inside
    the pulse)."""
    prob = W.softcore_3d(n=512, steps=SOFTCORE_STEPS, precision="c128")
    prob.t0 = 9.5
    psi0 = oracle_mod.gaussian(prob.grid, prob.init.center, prob.init.sigma, prob.init.k)
    ref = oracle_mod.propagate(prob.grid, prob.pot, psi0, SOFTCORE_STEPS, t0=prob.t0)
    del psi0
    return ref


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
def test_softcore_512_steps_elementwise(S, W, softcore_512_oracle, precision):
    """512^3 soft-core: 3 steps from t0 = 9.5, every point against the oracle.
    The FP32 state runs in the launch configuration the throughput benchmark
    times: 8 x slabs on two streams, potential and middle passes in variant
    0, the kinetic pass in variant 1 (8 values per thread); the two
    first-axis passes between the steps are the steady two-transform
    kernel."""
    prob = W.softcore_3d(n=512, steps=SOFTCORE_STEPS, precision=precision)
    prob.t0 = 9.5
    try:
        if precision == "c64":
            S.tune_set(False, "c64", 9, True, "potential", 0)
            S.tune_set(False, "c64", 9, True, "fft", 0)
            S.tune_set(False, "c64", 9, False, "kinetic", 1)
        s = S.from_problem(prob)
        if precision != "c128":
            s.set_slabs(8)
        s.propagate(SOFTCORE_STEPS)
        got = s.get_state("c128")
        norm = s.observables(1)["norm"]
        s.close()
    finally:
        S.tune_clear()
    err = rel_l2(got, softcore_512_oracle)
    print(f"512^3 softcore {precision} x {SOFTCORE_STEPS} steps: rel_l2 vs oracle {err:.3e}, "
          f"norm drift {abs(norm - 1):.2e}")
    assert err <= (1e-10 if precision == "c128" else 1e-4)
    assert abs(norm - 1.0) <= (1e-12 if precision == "c128" else 1e-5)


def test_softcore_512_full_length_fp32_vs_fp64(S, W):
    """The FP32 state after the stated 2000 steps against the FP64 state
    (FP64 pinned to the oracle above and at smaller sizes): rel-L2 <= 1e-4,
    norm drift <= 1e-5."""
    import torch

    prob = W.softcore_3d(n=512, steps=2000)
    a = S.from_problem(prob, precision="c64")
    b = S.from_problem(prob, precision="c128")
    for s in (a, b):
        s.propagate(2000)
        s.synchronize()
    x = torch.view_as_real(a.state_tensor()).double()
    y = torch.view_as_real(b.state_tensor())
    rel = float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y))
    n32, n64 = a.observables(1)["norm"], b.observables(1)["norm"]
    print(f"512^3 x 2000: rel_l2(f32, f64) = {rel:.3e}, norm drift f32 {abs(n32 - 1):.3e}, f64 {abs(n64 - 1):.3e}")
    a.close()
    b.close()
    assert rel <= 1e-4
    assert abs(n32 - 1.0) <= 1e-5
    assert abs(n64 - 1.0) <= 1e-12


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_softcore_512_reversible(S, W, precision):
    """50 steps forward from t0 = 9, then 50 steps with -dt from the reached
    time, return to the start (the trapezoid sampling makes the backward step
    the exact inverse)."""
    prob = W.softcore_3d(n=512, steps=50, precision=precision)
    prob.t0 = 9.0
    f = S.from_problem(prob)
    start = f.get_state("c128")
    f.propagate(50)
    t, _ = f.time()
    mid = f.get_state("c128")
    f.close()
    back = W.softcore_3d(n=512, steps=50, precision=precision)
    back.grid.dt = -prob.grid.dt
    g = S.Simulation(back.grid, back.pot, precision)
    g.set_state(mid, t0=t)
    del mid
    g.propagate(50)
    end = g.get_state("c128")
    g.close()
    assert rel_l2(end, start) <= (1e-12 if precision == "c128" else 1e-5)


def test_modulated_trap_1024_mean_position_classical(S, W):
    """Full 2D workload (1024^2, 2000 steps, FP64): for a quadratic potential
    the mean position follows the classical kick-drift-kick trajectory."""
    prob = W.modulated_trap_2d()
    s = S.from_problem(prob)
    x, p = np.array([3.0, -2.0]), np.array([0.0, 1.0])
    dt = prob.grid.dt
    force = lambda q, t: -np.array([(1 + 0.3 * math.cos(2 * t)) * q[0], (1 - 0.3 * math.cos(2 * t)) * q[1]])
    for n in range(2000):
        p = p + 0.5 * dt * force(x, n * dt)
        x = x + dt * p
        p = p + 0.5 * dt * force(x, (n + 1) * dt)
    s.propagate(2000)
    o = s.observables()
    s.close()
    assert abs(o["norm"] - 1.0) <= 1e-12
    assert abs(o["x"] - x[0]) <= 1e-9 and abs(o["y"] - x[1]) <= 1e-9


@pytest.fixture(scope="module")
def modulated_trap_oracle(W, oracle_mod):
    """The oracle's state of the full 2D workload: 1024^2, 2000 steps."""
    prob = W.modulated_trap_2d()
    psi0 = oracle_mod.gaussian(prob.grid, prob.init.center, prob.init.sigma, prob.init.k)
    return oracle_mod.propagate(prob.grid, prob.pot, psi0, prob.steps, t0=prob.t0)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_modulated_trap_1024_full_length_vs_oracle(S, W, modulated_trap_oracle, precision):
    """The full 2D workload (1024^2 on [-32, 32)^2, 2000 steps from the
    Gaussian) element by element against the oracle: 1e-10 for the FP64
    state; 1e-4 and norm drift 1e-5 for the FP32 state."""
    prob = W.modulated_trap_2d(precision=precision)
    s = S.from_problem(prob)
    s.propagate(prob.steps)
    got = s.get_state("c128")
    norm = s.observables(1)["norm"]
    s.close()
    err = rel_l2(got, modulated_trap_oracle)
    print(f"1024^2 x 2000 {precision}: rel_l2 vs oracle {err:.3e}, norm drift {abs(norm - 1):.2e}")
    assert err <= (1e-10 if precision == "c128" else 1e-4)
    assert abs(norm - 1.0) <= (1e-12 if precision == "c128" else 1e-5)


def test_modulated_trap_1024_fp32_parity_with_fp64(S, W):
    """Full 2D workload: the FP32 state within 1e-4 of the FP64 state, FP32
    norm drift within 1e-5."""
    prob = W.modulated_trap_2d()
    ref = S.from_problem(prob, precision="c128")
    ref.propagate(2000)
    r = ref.get_state("c128")
    ref.close()
    s = S.from_problem(prob, precision="c64")
    s.propagate(2000)
    g = s.get_state("c128")
    n = s.observables(1)["norm"]
    s.close()
    assert rel_l2(g, r) <= 1e-4
    assert abs(n - 1.0) <= 1e-5


def paul_leapfrog(W, prob, steps):
    d2 = 2 * 1.6e-3 ** 2
    amp = np.array([1.0, 1.0, -2.0]) * W.E_CHARGE_SI * 200.0 / (2 * d2)
    omega = 2 * math.pi * 18e6
    force = lambda x, t: -2 * amp * math.cos(omega * t) * x
    return leapfrog(np.array(prob.init.center), np.array(prob.init.k) * prob.grid.hbar, steps, prob.grid.dt,
                    0.0, force, mass=prob.grid.mass)


def test_paul_trap_512_fp64_classical(S, W):
    """Section 4.2 at full size (512^3, SI units), FP64: <x>, <y>, <z> follow
    the classical kick-drift-kick map every 250 steps for 2000 steps."""
    prob = W.paul_trap_3d(n=512, steps=2000, precision="c128")
    xs = paul_leapfrog(W, prob, 2000)
    s = S.from_problem(prob)
    for c in range(8):
        s.propagate(250)
        o = s.observables(0x0F)
        want = xs[250 * (c + 1)]
        got = np.array([o["x"], o["y"], o["z"]])
        assert np.all(np.abs(got - want) <= 1e-18), (c, got, want)  # metres
        assert abs(o["norm"] - 1.0) <= 1e-12
    s.close()


def test_paul_trap_512_fp32_full_length(S, W):
    """Section 4.2 at full size and length (512^3, 18500 steps), FP32 state:
    the trajectory within 1e-4 of the packet width of the classical map,
    norm drift <= 1e-5."""
    prob = W.paul_trap_3d(n=512, steps=18500, precision="c64")
    xs = paul_leapfrog(W, prob, 18500)
    s = S.from_problem(prob)
    worst = 0.0
    done = 0
    for n in [1850] * 10:
        s.propagate(n)
        done += n
        o = s.observables(0x0F)
        err = np.abs(np.array([o["x"], o["y"], o["z"]]) - xs[done])
        worst = max(worst, float(err.max()))
    s.close()
    print(f"Paul trap 512^3 x 18500 FP32: max |<x> - classical| = {worst:.3e} m, norm drift {abs(o['norm'] - 1):.2e}")
    assert worst <= 1e-4 * 3.7e-8
    assert abs(o["norm"] - 1.0) <= 1e-5


def test_softcore_2048_fp32_vs_fp64(S, W):
    """The largest power-of-two cube that fits one MI355X in both precisions
    at once: 2048^3 (64 GiB FP32 state, 128 GiB FP64 state) on [-160, 160)^3,
    the soft-core workload at its own spacing, 3 steps through the pulse.
    The FP32 state agrees with the FP64 state point by point (rel-L2 within
    1e-5, compared plane block by plane block on the device) and both keep
    their norms."""
    import torch

    need = S.state_bytes(W.softcore_3d(n=2048).grid, "c64") + S.state_bytes(W.softcore_3d(n=2048).grid, "c128")
    torch.cuda.empty_cache()  # blocks torch keeps cached count as used
    free, _ = torch.cuda.mem_get_info()
    if free < need + (8 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    prob = W.softcore_3d(n=2048, steps=3, half_width=160.0)
    prob.t0 = 9.5
    a = S.from_problem(prob, precision="c64")
    b = S.from_problem(prob, precision="c128")
    for s in (a, b):
        s.propagate(3)
        s.synchronize()
    x, y = a.state_tensor(), b.state_tensor()
    num = den = 0.0
    for p in range(0, 2048, 64):
        yd = torch.view_as_real(y[p:p + 64])
        d = torch.view_as_real(x[p:p + 64]).double() - yd
        num += float(torch.sum(d * d))
        den += float(torch.sum(yd * yd))
        del d, yd
    rel = (num / den) ** 0.5
    n32, n64 = a.observables(1)["norm"], b.observables(1)["norm"]
    print(f"2048^3 x 3: rel_l2(f32, f64) = {rel:.3e}, norm drift f32 {abs(n32 - 1):.2e}, f64 {abs(n64 - 1):.2e}")
    a.close()
    b.close()
    del x, y
    torch.cuda.empty_cache()
    assert rel <= 1e-5
    assert abs(n32 - 1.0) <= 1e-6 and abs(n64 - 1.0) <= 1e-12


def test_softcore_512_slabs_and_cache_hints_bit_identical(S, W):
    """At 512^3 the state is streamed with non-temporal hints, differently
    for one slab and for several: the results are the same bits."""
    prob = W.softcore_3d(n=512, steps=3, precision="c64")
    prob.t0 = 9.0
    out = []
    for count in (1, 4, 16):
        s = S.from_problem(prob)
        s.set_slabs(count)
        s.propagate(3)
        out.append(s.get_state("c64"))
        s.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_softcore_512_observe_fused_equals_separate(S, W, precision):
    """At full size the closing pass's moments (16384 workgroup rows in FP32)
    equal a propagation followed by a separate reduction, to the order of
    FP64 summation, and the states are the same bits."""
    prob = W.softcore_3d(n=512, steps=0, precision=precision)
    prob.t0 = 9.5
    a, b = S.from_problem(prob), S.from_problem(prob)
    mask = S.OBS_NORM | S.OBS_MOMENTS
    a.propagate(3)
    want = a.observables(mask)
    have = b.propagate_observe(3, mask)
    same = np.array_equal(a.state_tensor().cpu().numpy(), b.state_tensor().cpu().numpy())
    a.close()
    b.close()
    assert same
    scale = max(1.0, max(abs(v) for v in want.values()))
    for k, v in want.items():
        assert abs(have[k] - v) <= 1e-13 * scale, (k, have[k], v)
