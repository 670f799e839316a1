"""The paper's printed example inputs (tests/golden/, each file citing its
section) against what the workloads and the oracle pins use: a typo in a
transcribed constant fails here, on the CPU."""
import math
import os

import pytest

from paper_1306_3247_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, value = line.split()
                out[key] = float(value)
    return out


def test_paul_trap_workload_carries_the_printed_inputs():
    gi = read_golden("paul_trap_inputs.txt")
    prob = W.paul_trap_3d()
    g = prob.grid
    n = int(gi["points_per_axis"])
    assert list(g.n) == [n, n, n]
    assert list(g.lo) == [gi["grid_lo_m"]] * 3 and list(g.hi) == [gi["grid_hi_m"]] * 3
    assert g.dt == gi["dt_s"] and prob.steps == int(gi["steps"])
    assert g.mass == gi["mass_kg"] and W.BA138_MASS_SI == gi["mass_kg"]
    assert list(prob.init.center) == [gi["x0_m"], gi["y0_m"], gi["z0_centre_m"]]
    assert list(prob.init.sigma) == [gi["sigma_x_m"], gi["sigma_y_m"], gi["sigma_z_m"]]
    momenta = [gi["px0_kg_m_per_s"], gi["py0_kg_m_per_s"], gi["pz0_kg_m_per_s"]]
    for k, p in zip(prob.init.k, momenta):
        assert k * g.hbar == pytest.approx(p, rel=1e-15, abs=0.0)
    # V = Z e (U0 + V0 cos(Omega t)) (x^2 + y^2 - 2 z^2) / (2 d^2),
    # d^2 = r0^2 + 2 z0^2: the x^2 coefficient of each axis.
    d2 = gi["r0_m"] ** 2 * (1.0 + 2.0 * gi["z0_sq_over_r0_sq"])
    q = gi["charge_number"] * W.E_CHARGE_SI / (2.0 * d2)
    for axis, f in ((0, 1.0), (1, 1.0), (2, -2.0)):
        b = prob.pot.b[axis]
        assert b.kind == "cos"
        assert b.A0 == pytest.approx(f * q * gi["U0_V"], abs=1e-30)
        assert b.A1 == pytest.approx(f * q * gi["V0_V"], rel=1e-14)
        assert b.omega == pytest.approx(2.0 * math.pi * gi["Omega_over_2pi_Hz"], rel=1e-15)
    for axis in range(3):
        assert prob.pot.a[axis].A0 == 0.0 and prob.pot.a[axis].A1 == 0.0


def test_morse_parameters_of_the_oracle_pin():
    gi = read_golden("co_morse_inputs.txt")
    # the oracle's Morse pin (tests/test_oracle_pins.py) uses D and a of CO
    import test_oracle_pins as pins

    assert pins.CO_MORSE_D == gi["D_au"] and pins.CO_MORSE_A == gi["a_au"]
    # the printed field is the pulse of a 1 ps, resonant drive: its envelope
    # spans tf - ti atomic units of time (1 a.u. = 2.418884e-17 s)
    assert (gi["tf_au"] - gi["ti_au"]) * 2.418884e-17 == pytest.approx(1e-12, rel=1e-4)
    # and the grid of the eigenstates is 7-smooth (4000 = 2^5 5^3), a length
    # the mixed-radix kernels take
    n = int(gi["grid_points"])
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    assert n == 1
