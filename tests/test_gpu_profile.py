"""Per-launch device timing (wp_profile_propagate): the timed run advances the
state exactly as wp_propagate does, and every launcher that a schedule uses
(single-workgroup 1D solve, split 1D passes, mixed-radix passes and solves,
power-of-two line passes with and without x slabs, waveform coefficients)
takes the dispatch-attached events, so each class reports its launches."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NSTEPS = 6


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


def case(W, name, precision):
    if name == "1d":
        return W.driven_ho_1d(n=1024, steps=0, precision=precision), 1
    if name == "1d_split":
        return W.driven_ho_1d(n=1 << 14, steps=0, precision=precision), 1
    if name == "1d_mixed":
        p = W.driven_ho_1d(n=1024, steps=0, precision=precision)
        p.grid.n = [840]
        return p, 1
    if name == "2d":
        return W.modulated_trap_2d(n=64, steps=0, precision=precision, half_width=8.0), 1
    if name == "2d_mixed":
        p = W.modulated_trap_2d(n=64, steps=0, precision=precision, half_width=8.0)
        p.grid.n = [48, 60]
        return p, 1
    if name == "3d":
        return W.softcore_3d(n=32, steps=0, precision=precision, half_width=5.0), 1
    if name == "3d_slabs":
        return W.softcore_3d(n=64, steps=0, precision=precision, half_width=5.0), 4
    raise ValueError(name)


def expected_counts(S, name, nslab):
    """Launches per class over NSTEPS steps in the default VKV order: one
    first-axis pass opening and one closing the run, one merged first-axis
    pass between consecutive steps, and the middle passes of every step
    once per x slab."""
    if name in ("1d", "1d_mixed"):
        return {"solve1d": 1}
    out = {"edge": 2, "axis0": NSTEPS - 1, "last": NSTEPS * nslab}
    if name.startswith("3d"):
        out["mid_fwd"] = NSTEPS * nslab
        out["mid_inv"] = NSTEPS * nslab
    return out


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("name", ["1d", "1d_split", "1d_mixed", "2d", "2d_mixed", "3d", "3d_slabs"])
def test_profile_matches_propagate(S, W, name, precision):
    prob, nslab = case(W, name, precision)
    print(f"profile case {name} {precision} grid {prob.grid.n[:prob.grid.ndim]}", flush=True)
    ref = S.from_problem(prob)
    got = S.from_problem(prob)
    if nslab > 1:
        ref.set_slabs(nslab)
        got.set_slabs(nslab)
    ref.propagate(NSTEPS)
    prof = got.profile_propagate(NSTEPS)
    a, b = ref.get_state("c128"), got.get_state("c128")
    ref.close()
    got.close()
    np.testing.assert_array_equal(b, a)
    counts = {k: c for k, (c, _) in prof.items()}
    want = expected_counts(S, name, nslab)
    coef = counts.pop("coef", 0)
    assert counts == want
    if name not in ("1d", "1d_mixed"):
        assert coef >= 1  # at least the table of the first steps
    for k, (c, ms) in prof.items():
        assert c > 0 and np.isfinite(ms) and ms > 0.0, (k, c, ms)


def test_profile_selected_classes(S, W):
    prob, _ = case(W, "3d", "c64")
    ref = S.from_problem(prob)
    got = S.from_problem(prob)
    ref.propagate(NSTEPS)
    prof = got.profile_propagate(NSTEPS, kinds=("axis0", "mid_inv"))
    a, b = ref.get_state("c128"), got.get_state("c128")
    ref.close()
    got.close()
    np.testing.assert_array_equal(b, a)
    assert set(prof) == {"axis0", "mid_inv"}
    assert prof["axis0"][0] == NSTEPS - 1 and prof["mid_inv"][0] == NSTEPS


def test_profile_then_propagate_continues(S, W):
    """A timed run and an ordinary run compose: the step counter and the
    potential's time advance through both."""
    prob, _ = case(W, "2d", "c128")
    ref = S.from_problem(prob)
    got = S.from_problem(prob)
    ref.propagate(2 * NSTEPS + 3)
    got.propagate(3)
    got.profile_propagate(NSTEPS)
    got.propagate(NSTEPS)
    a, b = ref.get_state("c128"), got.get_state("c128")
    ref.close()
    got.close()
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * np.abs(a).max())
