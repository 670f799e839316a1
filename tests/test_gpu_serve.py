"""Serving loop (paper_1306_3247_amd.serve): admission by HBM budget,
continuous batching, asynchronous retirement.  Every result served in the
mix equals the same solve run alone with the same split into propagate
calls, bit for bit; it agrees with the solve run alone in one call within
the FP32 tolerance, and FP64 requests agree with the oracle."""
import numpy as np
import pytest

from conftest import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


@pytest.fixture(scope="module")
def V():
    from paper_1306_3247_amd import serve

    return serve


def small_stream(W, count, rate, seed, precision="c64"):
    return W.serving_stream(count, rate, seed=seed, log2_1d=(8, 15), sizes_2d=(32, 64, 128),
                            sizes_3d=(16, 32), steps_range=(20, 300), precision=precision)


def alone(S, prob, chunks):
    s = S.from_problem(prob)
    for n in chunks:
        s.propagate(n)
    out = s.get_state(prob.precision if prob.precision == "c128" else "c64")
    s.close()
    return out


def test_served_equals_alone(S, W, V):
    reqs = small_stream(W, 40, 400.0, seed=11)
    rep = V.Server(tick_steps=48, graph_steps=4, keep_results=True).run(reqs)
    by_id = {r.rid: r for r in reqs}
    assert all(not s.rejected for s in rep.served)
    assert rep.batches >= 2  # membership changed while serving
    multi = 0
    for s in rep.served:
        prob = by_id[s.rid].problem
        assert sum(s.chunks) == prob.steps
        multi += len(s.chunks) > 1
        same_split = alone(S, prob, s.chunks)
        assert np.array_equal(s.result, same_split), (s.rid, prob.name, s.chunks)
        one_call = alone(S, prob, [prob.steps])
        assert rel_l2(s.result, one_call) <= 1e-4, (s.rid, prob.name)
    assert multi > 0


def test_served_fp64_matches_oracle(S, W, V, oracle_mod):
    reqs = small_stream(W, 8, 200.0, seed=12, precision="c128")
    rep = V.Server(tick_steps=32, graph_steps=0, keep_results=True).run(reqs)
    for s, r in zip(sorted(rep.served, key=lambda x: x.rid), sorted(reqs, key=lambda x: x.rid)):
        p = r.problem
        psi0 = oracle_mod.gaussian(p.grid, p.init.center, p.init.sigma, p.init.k)
        ref = oracle_mod.propagate(p.grid, p.pot, psi0, p.steps, t0=p.t0)
        assert rel_l2(s.result, ref) <= 1e-10, p.name


def test_admission_respects_budget_and_overlaps(S, W, V):
    """A budget that holds only a few solves: the resident bytes never exceed
    it, requests wait for memory, and solves still share the device."""
    reqs = small_stream(W, 24, float("inf"), seed=13)
    sizes = sorted(V.Server.request_bytes(r.problem) for r in reqs)
    budget = sizes[-1] + sizes[-2] + sizes[-3]
    rep = V.Server(budget_bytes=budget, tick_steps=40, graph_steps=0, keep_results=False).run(reqs)
    assert rep.peak_bytes <= budget
    assert all(not s.rejected for s in rep.served)
    done = rep.served
    assert max(s.admitted for s in done) > min(s.finished for s in done)  # some waited for memory
    overlap = any(a.admitted < b.finished and b.admitted < a.finished
                  for i, a in enumerate(done) for b in done[i + 1:])
    assert overlap


def test_late_arrivals_join_running_solves(S, W, V):
    """A request arriving while a long solve runs is admitted at the next
    tick, long before that solve ends (continuous batching, not a queue)."""
    long_p = W.driven_trap(2, 512, 0.1, 1.0, [0, 0], [0, 0], steps=4000, precision="c64")
    short_p = W.driven_trap(1, 4096, 0.05, 1.5, [1.0], [0.5], steps=100, precision="c64")
    reqs = [W.Request(0, 0.0, long_p), W.Request(1, 0.03, short_p)]
    rep = V.Server(tick_steps=64, graph_steps=8, keep_results=True).run(reqs)
    a, b = sorted(rep.served, key=lambda s: s.rid)
    assert b.admitted < a.finished and b.finished < a.finished
    assert np.array_equal(b.result, alone(S, short_p, b.chunks))
    assert np.array_equal(a.result, alone(S, long_p, a.chunks))


def test_oversized_request_rejected(S, W, V):
    big = W.driven_trap(2, 256, 0.1, 1.0, [0, 0], [0, 0], steps=10, precision="c64")
    small = W.driven_trap(1, 1024, 0.1, 1.0, [0.0], [0.0], steps=10, precision="c64")
    budget = V.Server.request_bytes(small) * 2
    rep = V.Server(budget_bytes=budget, tick_steps=8).run([W.Request(0, 0.0, big), W.Request(1, 0.0, small)])
    r = {s.rid: s for s in rep.served}
    assert r[0].rejected and not r[1].rejected
    assert np.isfinite(r[1].finished)
