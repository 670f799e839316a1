import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU runs")


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def leapfrog(x, p, steps, dt, t0, force, mass=1.0):
    """Kick (dt/2) at t_n, drift, kick (dt/2) at t_{n+1}; force(x, t)."""
    xs = [x.copy()]
    for n in range(steps):
        tn, tn1 = t0 + n * dt, t0 + (n + 1) * dt
        p = p + 0.5 * dt * force(x, tn)
        x = x + dt * p / mass
        p = p + 0.5 * dt * force(x, tn1)
        xs.append(x.copy())
    return np.array(xs)


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    return oracle
