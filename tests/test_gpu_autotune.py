"""Kernel variants and the autotuner (wp_autotune, wp_batch_autotune,
wp_tune_*): every variant computes the same values in the same order, so
results are bit-identical whichever variant the table selects; tuning
leaves states untouched and picks the fastest timed candidate."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KINDS = ("fft", "potential", "kinetic")


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


@pytest.fixture(autouse=True)
def clean_table(S):
    S.tune_clear()
    yield
    S.tune_clear()


def force_variant(S, precision, variant, batched=False):
    for lg in range(6, 11):
        for strided in (False, True):
            for k in KINDS:
                S.tune_set(batched, precision, lg, strided, k, variant)


def problems(W, precision):
    p3 = W.softcore_3d(n=64, steps=0, precision=precision, half_width=5.0)
    p3.t0 = 9.0
    p2 = W.modulated_trap_2d(n=64, steps=0, precision=precision, half_width=8.0)
    p2.grid.n = [256, 1024]
    p2b = W.modulated_trap_2d(n=512, steps=0, precision=precision, half_width=8.0)
    return [p3, p2, p2b]


def run(S, prob, nsteps=5):
    s = S.from_problem(prob)
    s.propagate(nsteps)
    out = s.get_state("c128")
    s.close()
    return out


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_variants_bit_identical(S, W, precision):
    variants = (0, 1, 2, 3) if precision == "c64" else (0, 2)
    for prob in problems(W, precision):
        ref = run(S, prob)
        for v in variants[1:]:
            force_variant(S, precision, v)
            got = run(S, prob)
            S.tune_clear()
            assert np.array_equal(got, ref), (prob.name, prob.grid.n, v)


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_autotune_picks_fastest_and_keeps_state(S, W, precision):
    prob = W.softcore_3d(n=128, steps=0, precision=precision, half_width=10.0)
    s = S.from_problem(prob)
    s.propagate(3)
    before = s.get_state("c128")
    times = s.autotune(reps=5)
    after = s.get_state("c128")
    assert np.array_equal(before, after)
    assert set(times) == {"axis0", "mid", "last", "slabs"}
    expect = {"axis0": (True, "potential"), "mid": (True, "fft"), "last": (False, "kinetic")}
    for cls, row in times.items():
        if cls == "slabs":
            continue
        assert row and all(ms > 0 for ms in row.values())
        strided, kind = expect[cls]
        chosen = S.tune_get(False, precision, 7, strided, kind)
        assert chosen in row and row[chosen] == min(row.values())
    # tuned passes give the same result
    s.propagate(4)
    got = s.get_state("c128")
    s.close()
    S.tune_clear()
    ref = S.from_problem(prob)
    ref.propagate(3)
    ref.propagate(4)
    assert np.array_equal(got, ref.get_state("c128"))
    ref.close()


def test_batch_autotune_restores_states_and_matches_alone(S, W):
    probs = [W.driven_trap(2, n, 0.05 * (i + 1), 1.0 + 0.1 * i, [0.5, -0.5], [0.2, 0.1], steps=0, precision=prec)
             for i, (n, prec) in enumerate([(128, "c64"), (256, "c64"), (512, "c64"), (128, "c128"), (256, "c128")])]
    p3 = W.softcore_3d(n=64, steps=0, precision="c64", half_width=5.0)
    probs.append(p3)
    sims = [S.from_problem(p) for p in probs]
    for s in sims:
        s.propagate(2)
    before = [s.get_state("c128") for s in sims]
    b = S.Batch(sims, graph_steps=4)
    b.autotune(reps=3)
    after = [s.get_state("c128") for s in sims]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    b.propagate(11)
    b.close()
    got = [s.get_state("c128") for s in sims]
    for s in sims:
        s.close()
    S.tune_clear()
    for p, g in zip(probs, got):
        s = S.from_problem(p)
        s.propagate(2)
        s.propagate(11)
        assert np.array_equal(g, s.get_state("c128")), p.name
        s.close()


def test_tune_set_rejects_out_of_range(S):
    with pytest.raises(S.WavepacketError):
        S.tune_set(False, "c64", 9, True, "potential", 4)
    with pytest.raises(S.WavepacketError):
        S.tune_set(False, "c64", 13, True, "potential", 1)


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_slabs_bit_identical(S, W, precision):
    """The middle passes of a 3D step run slab by slab: the same arithmetic
    for every slab count, in both orders."""
    for order in ("vkv", "kvk"):
        prob = W.softcore_3d(n=64, steps=0, precision=precision, half_width=5.0)
        prob.t0 = 9.0
        out = []
        for count in (1, 2, 8, 64):
            s = S.from_problem(prob, order=order)
            s.set_slabs(count)
            assert s.slabs() == count
            s.propagate(5)
            out.append(s.get_state("c128"))
            s.close()
        for o in out[1:]:
            assert np.array_equal(o, out[0]), order


def test_slabs_rejected_where_meaningless(S, W):
    p2 = W.modulated_trap_2d(n=64, steps=0, precision="c64")
    s = S.from_problem(p2)
    s.set_slabs(1)
    with pytest.raises(S.WavepacketError):
        s.set_slabs(2)
    s.close()
    p3 = W.softcore_3d(n=16, steps=0, precision="c64", half_width=3.0)
    s = S.from_problem(p3)
    for bad in (3, 32):
        with pytest.raises(S.WavepacketError):
            s.set_slabs(bad)
    s.close()


def test_autotune_picks_a_slab_count(S, W):
    prob = W.softcore_3d(n=128, steps=0, precision="c64", half_width=10.0)
    s = S.from_problem(prob)
    times = s.autotune(reps=4)
    assert "slabs" in times and set(times["slabs"]) == {1 << k for k in range(8)}
    assert s.slabs() == min(times["slabs"], key=times["slabs"].get)
    s.close()


@pytest.mark.parametrize("count", [2, 8])
def test_slab_streams_joined_before_caller_work(S, W, count):
    """Odd slabs run on the handle's second stream; work the caller queues
    on the handle's stream right after a propagation (no host wait) must see
    every slab of every step."""
    import torch

    prob = W.softcore_3d(n=128, steps=0, precision="c64", half_width=10.0)
    stream = torch.cuda.Stream()
    s = S.from_problem(prob, stream=stream)
    s.set_slabs(count)
    s.synchronize()
    copies = []
    with torch.cuda.stream(stream):
        for _ in range(3):
            s.propagate(4)
            copies.append(s.state_tensor().clone(memory_format=torch.contiguous_format))  # same stream
    stream.synchronize()
    final = s.get_state("c64")
    ref = S.from_problem(prob)
    ref.set_slabs(1)
    for i, c in enumerate(copies):
        ref.propagate(4)
        want = ref.get_state("c64")
        got = c.cpu().numpy().reshape(want.shape)
        assert np.array_equal(got, want), i
    assert np.array_equal(final, want)
    s.close()
    ref.close()
