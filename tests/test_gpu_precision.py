"""Precision guards of the FP32 state (complex64 storage, FP64 phase
arguments): the norm must not be biased step after step.

Every step is unitary (eq. splitop: each factor is a phase, and the Fourier
transform preserves the norm up to 1/N), so the FP32 path may change the norm
only by unbiased rounding.  A factor rounded to FP32 changes |psi| by the same
relative amount at every step; over the 2000 steps of the 512^3 workload a
bias of 5e-9 per step would already use the whole norm budget of 1e-5.  The
guard: on a soft-core grid at the workload's spacing, the norm changes by
less than 2e-9 per step on average, measured as the least-squares slope over
400 steps and as the total change.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


@pytest.mark.parametrize("precision", ["c64", "c64x"])
@pytest.mark.parametrize("n", [64, 128])
def test_fp32_norm_bias_per_step(S, W, n, precision):
    steps, every = 400, 25
    prob = W.softcore_3d(n=n, steps=steps, precision=precision, half_width=n * 0.078125)
    prob.t0 = 8.0  # through the pulse maximum at t = 10
    s = S.from_problem(prob)
    norms = [s.observables(1)["norm"]]
    for _ in range(steps // every):
        s.propagate(every)
        norms.append(s.observables(1)["norm"])
    s.close()
    k = np.arange(len(norms)) * every
    slope = float(np.polyfit(k, np.array(norms) - norms[0], 1)[0])
    total = (norms[-1] - norms[0]) / steps
    print(f"{n}^3 {precision}: norm slope {slope:.2e} per step, mean change {total:.2e} per step")
    assert abs(slope) < 2e-9
    assert abs(total) < 2e-9
