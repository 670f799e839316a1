"""GPU path (through the C ABI) against the FP64 CPU oracle, element by element.

Tolerances (relative L2 over all points, no phase alignment): 1e-10 for the
FP64 state, 1e-4 for the FP32 state; FP32 norm drift 1e-5.  Sizes are small
enough for the oracle to finish in seconds and include workgroups with fewer
lines than the kernel's tile (ragged tails).  Power-of-two line lengths 2 to
4096 appear on the contiguous axis and on strided axes, and 512 and 1024
(the lengths of the 3D and 2D throughput workloads) on every axis of 2D and
3D grids, in every precision.
"""
import numpy as np
import pytest

from conftest import rel_l2

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-4, "c64x": 1e-4}


def shape_id(shape):
    return "x".join(str(n) for n in shape)


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


def morse_dipole_1d(W, n, steps, precision):
    """Morse oscillator with a sin^2-envelope dipole drive (the form of Section 4.1)."""
    g = W.Grid(1, [n], [0.5], [6.5], mass=20.0, dt=0.05)
    p = W.Potential(v0_kind="morse", v0_par=(0.4, 1.2, 2.1, 0.0))
    p.s = W.const(1.0)
    p.a[0] = W.Wave("sin2_cos", A0=0.0, A1=-0.9 * 0.05, omega=0.3, ti=0.0, tf=4.0)
    p.c = W.Wave("sin2_cos", A0=0.0, A1=0.15 * 0.05, omega=0.3, ti=0.0, tf=4.0)
    return W.Problem("morse_1d", g, p, W.Gaussian([2.3], [0.5], [0.0]), steps, precision)


def run_both(S, oracle, prob, psi0=None, order="vkv"):
    s = S.Simulation(prob.grid, prob.pot, prob.precision, order=order)
    if psi0 is None:
        s.set_gaussian(prob.init.center, prob.init.sigma, prob.init.k, prob.t0)
        psi0 = oracle.gaussian(prob.grid, prob.init.center, prob.init.sigma, prob.init.k)
    else:
        s.set_state(psi0, prob.t0)
    s.propagate(prob.steps)
    got = s.get_state("c128")
    s.close()
    ref = oracle.propagate(prob.grid, prob.pot, psi0, prob.steps, t0=prob.t0,
                           order=oracle.ORDER_KVK if order == "kvk" else oracle.ORDER_VKV)
    return got, ref, psi0


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
@pytest.mark.parametrize("order", ["vkv", "kvk"])
@pytest.mark.parametrize("n", [2, 4, 8, 16, 64, 512, 1024, 8192])
def test_1d_random_state(S, W, oracle_mod, n, order, precision):
    prob = W.driven_ho_1d(n=n, steps=7, precision=precision)
    psi0 = W.random_state((n,), seed=n)
    psi0 /= np.linalg.norm(psi0)
    got, ref, _ = run_both(S, oracle_mod, prob, psi0, order)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
@pytest.mark.parametrize("order", ["vkv", "kvk"])
@pytest.mark.parametrize("n", [16384, 32768, 65536, 1 << 20])
def test_1d_split_random_state(S, W, oracle_mod, n, order, precision):
    """1D grids beyond the single-workgroup solver: the [n1][n2] split
    transform (n1 = n2 and n1 = 2 n2), up to the largest supported length."""
    prob = W.driven_ho_1d(n=n, steps=5, precision=precision)
    psi0 = W.random_state((n,), seed=n + 1)
    psi0 /= np.linalg.norm(psi0)
    got, ref, _ = run_both(S, oracle_mod, prob, psi0, order)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_1d_split_driven_trap(S, W, oracle_mod, precision):
    """The serving mix's largest 1D request shape: 2^16 points on [-20, 20),
    driven trap, 300 steps from a Gaussian."""
    prob = W.driven_trap(1, 65536, E0=0.15, omega=1.3, center=[1.5], k=[-0.5], steps=300,
                         precision=precision, half_width=20.0)
    got, ref, psi0 = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("v0", ["morse", "softcore"])
def test_1d_split_nonseparable(S, W, oracle_mod, v0, precision):
    """Per-point potentials on a split grid: the Morse oscillator and a 1D
    soft-core well."""
    prob = morse_dipole_1d(W, 16384, 40, precision)
    if v0 == "softcore":
        prob.grid.lo, prob.grid.hi = [-30.0], [30.0]
        prob.pot.v0_kind, prob.pot.v0_par = "softcore", (1.0, 2.0, 0.0, 0.0)
        prob.grid.mass = 1.0
        prob.init = W.Gaussian([0.0], [1.0], [0.5])
    got, ref, _ = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]


# Mixed-radix lengths (prime factors 2, 3, 5, 7): every radix and several
# factor orders, odd lengths, up to the 4096-point limit.
@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("order", ["vkv", "kvk"])
@pytest.mark.parametrize("n", [3, 5, 6, 7, 12, 15, 49, 105, 360, 2520, 3087, 4000])
def test_1d_mixed_random_state(S, W, oracle_mod, n, order, precision):
    prob = W.driven_ho_1d(n=n, steps=6, precision=precision)
    psi0 = W.random_state((n,), seed=n + 3)
    psi0 /= np.linalg.norm(psi0)
    got, ref, _ = run_both(S, oracle_mod, prob, psi0, order)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
@pytest.mark.parametrize("order", ["vkv", "kvk"])
@pytest.mark.parametrize("shape", [(6, 10), (15, 64), (64, 21), (360, 120), (7, 49), (3, 4096)])
def test_2d_mixed_random_state(S, W, oracle_mod, shape, order, precision):
    prob = W.modulated_trap_2d(n=4, steps=4, precision=precision)
    prob.grid.n = list(shape)
    psi0 = W.random_state(shape, seed=5 + sum(shape))
    psi0 /= np.linalg.norm(psi0)
    got, ref, _ = run_both(S, oracle_mod, prob, psi0, order)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
@pytest.mark.parametrize("order", ["vkv", "kvk"])
@pytest.mark.parametrize("shape", [(6, 10, 14), (3, 5, 7), (30, 24, 20), (16, 9, 32)])
def test_3d_mixed_random_state(S, W, oracle_mod, shape, order, precision):
    prob = W.softcore_3d(n=4, steps=3, precision=precision, half_width=6.0)
    prob.grid.n = list(shape)
    prob.t0 = 9.0
    psi0 = W.random_state(shape, seed=11 + sum(shape))
    psi0 /= np.linalg.norm(psi0)
    got, ref, _ = run_both(S, oracle_mod, prob, psi0, order)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_mixed_gaussian_physics(S, W, oracle_mod, precision):
    """A Gaussian in the modulated trap on a 360 x 375 grid (2^3 3^2 5 and
    3 5^3 points), 200 steps, against the oracle; observables too."""
    prob = W.modulated_trap_2d(n=4, steps=200, precision=precision, half_width=8.0)
    prob.grid.n = [360, 375]
    got, ref, psi0 = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]
    t = prob.t0 + prob.steps * prob.grid.dt
    if precision != "c128":  # the values an FP32 state holds
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
        ref = ref.astype(np.complex64).astype(np.complex128)
    s = S.Simulation(prob.grid, prob.pot, precision)
    s.set_state(psi0, t0=prob.t0)
    s.store_reference()
    s.set_state(ref, t0=t)
    o = s.observables(S.OBS_ALL_EXT)
    s.close()
    want = oracle_all(oracle_mod, prob, ref, t, psi0)
    scale = max(1.0, max(abs(v) for v in want.values()))
    for k in KEYS:
        tol = 2e-6 if (k == "energy" and precision != "c128") else 1e-12
        assert abs(o[k] - want[k]) <= tol * scale, (k, o[k], want[k])


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("n,v0", [(1000, "morse"), (2187, "softcore")])
def test_1d_mixed_nonseparable(S, W, oracle_mod, n, v0, precision):
    """Per-point potentials through the mixed-radix solver: the Morse
    oscillator on 1000 = 2^3 5^3 points and a soft-core well on 3^7."""
    prob = morse_dipole_1d(W, n, 40, precision)
    if v0 == "softcore":
        prob.grid.lo, prob.grid.hi = [-30.0], [30.0]
        prob.pot.v0_kind, prob.pot.v0_par = "softcore", (1.0, 2.0, 0.0, 0.0)
        prob.grid.mass = 1.0
        prob.init = W.Gaussian([0.0], [1.0], [0.5])
    got, ref, _ = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_paul_trap_mixed_grid(S, W, oracle_mod, precision):
    """The Section 4.2 Paul trap (SI units) on a 60 x 48 x 45 grid at the
    paper's spacing through the mixed-radix passes."""
    prob = W.paul_trap_3d(n=64, steps=20, precision=precision, half_width=1.25e-7)
    dx = 2.5e-7 / 64
    prob.grid.n = [60, 48, 45]
    prob.grid.lo = [-30 * dx, -24 * dx, -22.5 * dx]
    prob.grid.hi = [30 * dx, 24 * dx, 22.5 * dx]
    got, ref, _ = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("graph_steps", [0, 4])
def test_mixed_members_in_a_batch(S, W, graph_steps):
    """Members on mixed-length grids (1D, 2D, 3D, both precisions) advance in
    a batch beside power-of-two members with their own launches: every
    result equals its own wp_propagate result bit for bit."""
    probs = []
    p = W.modulated_trap_2d(n=4, steps=0, precision="c64", half_width=8.0)
    p.grid.n = [60, 72]
    probs.append(p)
    p = W.softcore_3d(n=4, steps=0, precision="c128", half_width=5.0)
    p.grid.n = [24, 20, 30]
    p.t0 = 9.0
    probs.append(p)
    probs.append(W.driven_ho_1d(n=1000, steps=0, precision="c64"))
    probs.append(W.modulated_trap_2d(n=64, steps=0, precision="c64", half_width=8.0))
    probs.append(W.driven_ho_1d(n=512, steps=0, precision="c128"))
    sims = [S.from_problem(q) for q in probs]
    refs = [S.from_problem(q) for q in probs]
    b = S.Batch(sims, graph_steps=graph_steps)
    b.propagate(11)
    b.propagate(6)
    for r in refs:
        r.propagate(11)
        r.propagate(6)
    for q, x, r in zip(probs, sims, refs):
        prec = "c128" if q.precision == "c128" else "c64"
        assert np.array_equal(x.get_state(prec), r.get_state(prec)), q.name
        assert x.time() == r.time()
    b.close()
    for x in sims + refs:
        x.close()


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
def test_1d_morse(S, W, oracle_mod, precision):
    prob = morse_dipole_1d(W, 512, 100, precision)
    got, ref, _ = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]


def test_driven_ho_1d_full_length(S, W, oracle_mod):
    prob = W.driven_ho_1d()  # 1024 points, 1000 steps, FP64
    got, ref, _ = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= 1e-10


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
@pytest.mark.parametrize("order", ["vkv", "kvk"])
# 512 and 1024 points on the strided first axis (the potential pass; 1024
# is the modulated trap's x axis: twiddles read from global memory) and on
# the contiguous last axis (the kinetic pass), with full and partial tiles.
@pytest.mark.parametrize("shape", [(2, 2), (4, 8), (16, 256), (128, 32), (64, 64), (8, 4096), (4096, 4),
                                   (512, 8), (512, 32), (1024, 8), (1024, 2), (8, 512), (2, 1024),
                                   (16, 1024), (2048, 4), (4, 2048), (256, 16), (32, 128)], ids=shape_id)
def test_2d_random_state(S, W, oracle_mod, shape, order, precision):
    prob = W.modulated_trap_2d(n=4, steps=5, precision=precision)
    prob.grid.n = list(shape)
    psi0 = W.random_state(shape, seed=sum(shape))
    psi0 /= np.linalg.norm(psi0)
    got, ref, _ = run_both(S, oracle_mod, prob, psi0, order)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
@pytest.mark.parametrize("order", ["vkv", "kvk"])
# 512 to 4096 points on each of the three axes: the first-axis potential
# pass (padded planes), the middle-axis FFT pass (strided) and the last-axis
# kinetic pass (contiguous), with full and partial tiles.
@pytest.mark.parametrize("shape", [(2, 4, 2), (8, 8, 8), (16, 64, 8), (32, 32, 32), (4, 2, 1024),
                                   (512, 4, 8), (512, 2, 2), (1024, 2, 4), (8, 512, 4), (4, 1024, 2),
                                   (8, 4, 512), (2, 8, 1024), (2048, 2, 2), (2, 2048, 4), (4, 2, 2048),
                                   (4096, 2, 2), (2, 4096, 2), (2, 2, 4096)], ids=shape_id)
def test_3d_random_state(S, W, oracle_mod, shape, order, precision):
    prob = W.softcore_3d(n=4, steps=4, precision=precision, half_width=6.0)
    prob.grid.n = list(shape)
    prob.t0 = 9.0  # inside the pulse
    psi0 = W.random_state(shape, seed=7 + sum(shape))
    psi0 /= np.linalg.norm(psi0)
    got, ref, _ = run_both(S, oracle_mod, prob, psi0, order)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
def test_modulated_trap_2d_scaled(S, W, oracle_mod, precision):
    """Modulated trap at the full spacing (1/16) on a 256^2 box, 400 steps."""
    prob = W.modulated_trap_2d(n=256, steps=400, precision=precision, half_width=8.0)
    got, ref, psi0 = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]
    drift = abs(np.linalg.norm(got) - np.linalg.norm(psi0)) / np.linalg.norm(psi0)
    assert drift <= (1e-12 if precision == "c128" else 1e-5)


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
def test_softcore_3d_scaled(S, W, oracle_mod, precision):
    """Soft-core atom at the full spacing (0.15625) on a 64^3 box through the pulse."""
    prob = W.softcore_3d(n=64, steps=60, precision=precision, half_width=5.0)
    prob.t0 = 9.5
    got, ref, psi0 = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
def test_paul_trap_si_scaled(S, W, oracle_mod, precision):
    """The Section 4.2 Paul trap (SI units) at the paper's spacing on a 64^3
    box, 40 steps, every point."""
    prob = W.paul_trap_3d(n=64, steps=40, precision=precision, half_width=1.25e-7)
    got, ref, _ = run_both(S, oracle_mod, prob)
    assert rel_l2(got, ref) <= TOL[precision]


def observable_problem(W, which, precision):
    if which == "1d":
        prob = morse_dipole_1d(W, 1024, 30, precision)
        prob.t0 = 1.0
    elif which == "1d_split":
        prob = W.driven_trap(1, 32768, E0=0.1, omega=1.0, center=[-2.0], k=[1.0], steps=30,
                             precision=precision, half_width=20.0)
        prob.t0 = 1.0
    elif which == "2d":
        prob = W.modulated_trap_2d(n=128, steps=30, precision=precision, half_width=8.0)
    else:
        prob = W.softcore_3d(n=32, steps=10, precision=precision, half_width=5.0)
        prob.t0 = 9.0
    return prob


def oracle_all(oracle_mod, prob, psi, t, psi_ref):
    """Every observable from the oracle: Table 3 widths from its moments,
    the autocorrelation from its inner product."""
    ref = oracle_mod.observables(prob.grid, prob.pot, psi, t)
    for a, m, m2 in (("sx", "x", "x2"), ("sy", "y", "y2"), ("sz", "z", "z2")):
        ref[a] = ref[m2] - ref[m] ** 2
    ref["autocorrelation"] = abs(oracle_mod.inner(prob.grid, psi_ref, psi)) ** 2
    return ref


KEYS = ("norm", "x", "y", "z", "x2", "y2", "z2", "energy", "sx", "sy", "sz", "autocorrelation")


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
@pytest.mark.parametrize("which", ["1d", "1d_split", "2d", "3d"])
def test_observables_of_oracle_state(S, W, oracle_mod, which, precision):
    """The reductions alone: the oracle's propagated state is loaded into the
    handle, with the oracle's initial state as the autocorrelation reference."""
    prob = observable_problem(W, which, precision)
    psi0 = oracle_mod.gaussian(prob.grid, prob.init.center, prob.init.sigma, prob.init.k)
    psi = oracle_mod.propagate(prob.grid, prob.pot, psi0, prob.steps, t0=prob.t0)
    if precision != "c128":
        # The FP32 state holds the values rounded to complex64: the oracle
        # evaluates the observables of exactly those values.
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
        psi = psi.astype(np.complex64).astype(np.complex128)
    t = prob.t0 + prob.steps * prob.grid.dt
    s = S.Simulation(prob.grid, prob.pot, precision)
    s.set_state(psi0, t0=prob.t0)
    s.store_reference()
    s.set_state(psi, t0=t)
    got = s.observables(S.OBS_ALL_EXT)
    s.close()
    ref = oracle_all(oracle_mod, prob, psi, t, psi0)
    scale = max(1.0, max(abs(v) for v in ref.values()))
    # Every reduction is FP64 over the same values; only the kinetic part of
    # the energy of an FP32 state goes through a device transform whose
    # result is stored in FP32 (relative 6e-8 per value).
    for k in KEYS:
        tol = 2e-6 if (k == "energy" and precision != "c128") else 1e-12
        assert abs(got[k] - ref[k]) <= tol * scale, (k, got[k], ref[k])


@pytest.mark.parametrize("precision", ["c128", "c64", "c64x"])
@pytest.mark.parametrize("which", ["1d", "1d_split", "2d", "3d"])
def test_observables_after_propagation(S, W, oracle_mod, which, precision):
    """End to end: device propagation and reductions against the oracle's
    propagation and reductions (tolerance of the state parity)."""
    prob = observable_problem(W, which, precision)
    s = S.from_problem(prob)
    s.store_reference()
    s.propagate(prob.steps)
    got = s.observables(S.OBS_ALL_EXT)
    t, n = s.time()
    s.close()
    assert n == prob.steps
    assert t == prob.t0 + prob.steps * prob.grid.dt
    psi0 = oracle_mod.gaussian(prob.grid, prob.init.center, prob.init.sigma, prob.init.k)
    psi = oracle_mod.propagate(prob.grid, prob.pot, psi0, prob.steps, t0=prob.t0)
    ref = oracle_all(oracle_mod, prob, psi, t, psi0)
    scale = max(1.0, max(abs(v) for v in ref.values()))
    tol = 1e-9 if precision == "c128" else 2e-4
    for k in KEYS:
        assert abs(got[k] - ref[k]) <= tol * scale, (k, got[k], ref[k])


@pytest.mark.parametrize("phi_dtype", ["complex64", "complex128"])
@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_inner_product(S, W, oracle_mod, precision, phi_dtype):
    """<phi|psi> with a seeded phi on the device, against the oracle."""
    import torch

    prob = W.modulated_trap_2d(n=64, steps=0, precision=precision, half_width=8.0)
    prob.grid.n = [64, 128]
    psi = W.random_state((64, 128), seed=3)
    phi = W.random_state((64, 128), seed=4)
    if phi_dtype == "complex64":
        phi = phi.astype(np.complex64).astype(np.complex128)
    if precision == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    s = S.Simulation(prob.grid, prob.pot, precision)
    s.set_state(psi)
    got = s.inner(torch.from_numpy(phi.astype(phi_dtype)).cuda())
    s.close()
    ref = oracle_mod.inner(prob.grid, phi, psi)
    assert abs(got - ref) <= 1e-12 * abs(ref) + 1e-13


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("Z", [2.0, 50.0, 5000.0])
def test_phase_argument_regimes(S, W, oracle_mod, Z, precision):
    """Per-step phases of |theta| < 1/16, < pi/4 and well beyond (soft-core
    strength Z with dt = 0.01): every evaluation branch against the oracle."""
    prob = W.softcore_3d(n=16, steps=3, precision=precision, half_width=4.0)
    prob.pot.v0_par = (Z, 1.0, 0.0, 0.0)
    psi0 = W.random_state((16, 16, 16), seed=int(Z))
    psi0 /= np.linalg.norm(psi0)
    got, ref, _ = run_both(S, oracle_mod, prob, psi0)
    assert rel_l2(got, ref) <= TOL[precision]
