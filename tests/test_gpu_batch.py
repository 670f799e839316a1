"""Batched propagation (wp_batch_*): each solve advanced in a batch equals the
same solve advanced alone, for mixed sizes, dimensions, precisions, start
times and step counters, with direct launches and with replayed graphs."""
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


def mixed_problems(W):
    rng = np.random.default_rng(7)
    out = []
    specs = [(1, 256, "c128"), (1, 1024, "c64"), (2, 64, "c128"), (2, 128, "c64"), (2, 256, "c64x"),
             (2, 128, "c128"), (3, 32, "c64"), (3, 16, "c128"), (2, 512, "c64"), (1, 2048, "c64x"),
             (1, 16384, "c64"), (1, 65536, "c128"), (2, 2048, "c64")]
    for i, (ndim, n, prec) in enumerate(specs):
        p = W.driven_trap(ndim, n, E0=rng.uniform(0.01, 0.2), omega=rng.uniform(0.5, 2.0),
                          center=rng.uniform(-3, 3, ndim), k=rng.uniform(-1, 1, ndim), steps=0,
                          precision=prec, half_width=16.0 if ndim > 1 else 20.0)
        p.t0 = 0.37 * i  # different start times
        out.append(p)
    # one non-separable member: the soft-core atom on a small box
    q = W.softcore_3d(n=32, steps=0, precision="c64", half_width=5.0)
    q.t0 = 9.0
    out.append(q)
    return out


def split(nsteps, chunks):
    per = nsteps // chunks
    return [per] * (chunks - 1) + [nsteps - per * (chunks - 1)]


def run_alone(S, probs, pre, nsteps, chunks=1):
    res = []
    for p, k in zip(probs, pre):
        s = S.from_problem(p)
        s.propagate(k)
        for n in split(nsteps, chunks):
            s.propagate(n)
        res.append(s.get_state("c128"))
        s.close()
    return res


def run_batch(S, probs, pre, nsteps, graph_steps, chunks=1):
    sims = [S.from_problem(p) for p in probs]
    for s, k in zip(sims, pre):
        s.propagate(k)  # members start from different step counters
    b = S.Batch(sims, graph_steps=graph_steps)
    for n in split(nsteps, chunks):
        b.propagate(n)
    b.close()
    out = [s.get_state("c128") for s in sims]
    times = [s.time() for s in sims]
    for s in sims:
        s.close()
    return out, times


@pytest.mark.parametrize("graph_steps,nsteps,chunks", [(0, 13, 1), (8, 21, 1), (4, 17, 2), (0, 70, 1), (64, 150, 1),
                                                      (0, 1, 1), (5, 2, 1)])
def test_batch_equals_alone(S, W, graph_steps, nsteps, chunks):
    """Bit for bit: the batch runs the same kernels in the same order per
    solve, whatever the graph length."""
    probs = mixed_problems(W)
    pre = [i % 3 for i in range(len(probs))]
    alone = run_alone(S, probs, pre, nsteps, chunks)
    batch, times = run_batch(S, probs, pre, nsteps, graph_steps, chunks)
    for i, (a, b) in enumerate(zip(alone, batch)):
        assert np.array_equal(a, b), (i, probs[i].name, rel_l2(b, a))
    for p, k, (t, n) in zip(probs, pre, times):
        assert n == k + nsteps
        assert t == p.t0 + (k + nsteps) * p.grid.dt


def test_batch_members_match_oracle(S, W, oracle_mod):
    probs = [p for p in mixed_problems(W) if p.precision == "c128"]
    batch, _ = run_batch(S, probs, [0] * len(probs), 9, graph_steps=4)
    for p, got in zip(probs, batch):
        psi0 = oracle_mod.gaussian(p.grid, p.init.center, p.init.sigma, p.init.k)
        ref = oracle_mod.propagate(p.grid, p.pot, psi0, 9, t0=p.t0)
        assert rel_l2(got, ref) <= 1e-10, p.name


def test_batch_rejects_bad_input(S, W):
    p = W.driven_trap(2, 32, 0.1, 1.0, [0, 0], [0, 0], steps=0)
    s = S.from_problem(p)
    s.set_order("kvk")
    with pytest.raises(S.WavepacketError):
        S.Batch([s])
    s.close()


def test_zero_steps_are_no_ops(S, W):
    """propagate(0) leaves state, time and counters alone, alone and batched."""
    p = W.driven_trap(2, 64, 0.1, 1.0, [0.5, 0.0], [0.0, 0.3], steps=0, precision="c64")
    s = S.from_problem(p)
    s.propagate(3)
    before = s.get_state("c128")
    s.propagate(0)
    b = S.Batch([s], graph_steps=4)
    b.propagate(0)
    b.close()
    assert np.array_equal(s.get_state("c128"), before)
    assert s.time() == (p.t0 + 3 * p.grid.dt, 3)
    s.close()


def test_graph_replays_each_match_eager(S, W):
    """Every replay of the batch's captured step sequence gives the eager
    result: three calls of 9 steps with 4-step graphs (two replays and the
    direct first and last steps per call), the states read back to the host
    and other work queued on the device between the calls, each compared bit
    for bit with members stepped alone to the same step count."""
    import torch

    probs = [W.driven_trap(2, 128, 0.1, 1.3, [0.5, -0.2], [0.3, 0.0], steps=0, precision="c64"),
             W.driven_trap(2, 256, 0.05, 0.7, [-1.0, 0.4], [0.0, -0.2], steps=0, precision="c128"),
             W.softcore_3d(n=32, steps=0, precision="c64", half_width=5.0)]
    probs[2].t0 = 9.0
    alone = [S.from_problem(p) for p in probs]
    sims = [S.from_problem(p) for p in probs]
    b = S.Batch(sims, graph_steps=4)
    scratch = torch.zeros(1 << 20, device="cuda")
    for call in range(3):
        b.propagate(9)
        scratch.add_(1.0)  # eager work of the program between replays
        torch.cuda.synchronize()
        for a, s in zip(alone, sims):
            a.propagate(9)
            assert np.array_equal(s.get_state("c128"), a.get_state("c128")), (call, s.precision)
            assert s.time() == a.time()
    b.close()
    for s in alone + sims:
        s.close()
    assert float(scratch[0]) == 3.0
