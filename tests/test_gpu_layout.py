"""Storage of 3D power-of-two states: every x plane is followed by 16 unused
points (wp_state_pitch).  Host copies, the device view and the inner
product see only the grid's points, and no kernel reads or writes the
padding: with NaN written there, propagation, observables, the fused
moments and the autocorrelation give bit-identical results."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PAD = 16
GRIDS = [("c64", [64, 32, 16]), ("c128", [32, 64, 8]), ("c64x", [16, 16, 32])]


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


def problem(W, precision, n):
    prob = W.softcore_3d(n=16, steps=0, precision=precision, half_width=6.0)
    prob.grid.n = list(n)
    prob.t0 = 9.0  # inside the pulse
    return prob


def pad_positions(n, pitch):
    """Indices (in points) of the unused storage after each x plane."""
    plane = n[1] * n[2]
    return (np.arange(n[0])[:, None] * pitch + plane + np.arange(pitch - plane)[None, :]).ravel()


@pytest.mark.parametrize("precision,n", GRIDS)
def test_pitch_and_sizes(S, W, precision, n):
    prob = problem(W, precision, n)
    pitch = S.state_pitch(prob.grid, precision)
    assert pitch == n[1] * n[2] + PAD
    elem = 16 if precision == "c128" else 8
    assert S.state_bytes(prob.grid, precision) == n[0] * pitch * elem
    s = S.Simulation(prob.grid, prob.pot, precision)
    assert s.buffer.numel() == n[0] * pitch * elem
    assert tuple(s.state_tensor().shape) == tuple(n)
    s.close()


@pytest.mark.parametrize("precision,n", GRIDS)
def test_host_round_trip(S, W, precision, n):
    rng = np.random.default_rng(1306)
    psi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    prob = problem(W, precision, n)
    s = S.Simulation(prob.grid, prob.pot, precision)
    s.set_state(psi, 0.0)
    want = psi if precision == "c128" else psi.astype(np.complex64).astype(np.complex128)
    assert np.array_equal(s.get_state("c128"), want)
    store = "c128" if precision == "c128" else "c64"
    view = s.state_tensor().cpu().numpy()
    assert np.array_equal(view, s.get_state(store))
    s.close()


@pytest.mark.parametrize("precision,n", GRIDS)
def test_padding_never_touched(S, W, precision, n):
    import torch

    prob = problem(W, precision, n)
    ref = S.from_problem(prob)
    got = S.from_problem(prob)
    pitch = S.state_pitch(prob.grid, precision)
    cdt = torch.complex128 if precision == "c128" else torch.complex64
    flat = got.buffer.view(cdt)
    idx = torch.from_numpy(pad_positions(n, pitch)).to(flat.device)
    flat[idx] = complex(float("nan"), float("nan"))
    torch.cuda.synchronize()
    for s in (ref, got):
        s.store_reference()
        s.propagate(5)
    assert np.array_equal(got.get_state("c128"), ref.get_state("c128"))
    assert got.observables(S.OBS_ALL_EXT) == ref.observables(S.OBS_ALL_EXT)
    assert got.propagate_observe(3) == ref.propagate_observe(3)
    assert np.array_equal(got.get_state("c128"), ref.get_state("c128"))
    torch.cuda.synchronize()
    assert bool(torch.isnan(flat[idx].real).all()) and bool(torch.isnan(flat[idx].imag).all())
    ref.close()
    got.close()


@pytest.mark.parametrize("precision,n", GRIDS[:2])
def test_inner_takes_contiguous_phi(S, W, precision, n):
    import torch

    prob = problem(W, precision, n)
    s = S.from_problem(prob)
    s.propagate(3)
    rng = np.random.default_rng(7)
    phi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    dv = float(np.prod([(h - l) / m for l, h, m in zip(prob.grid.lo, prob.grid.hi, n)]))
    want = np.vdot(phi, s.get_state("c128")) * dv
    for dt in (torch.complex128, torch.complex64):
        p = torch.from_numpy(phi).to(dt).to("cuda")
        w = want if dt == torch.complex128 else np.vdot(phi.astype(np.complex64).astype(np.complex128),
                                                        s.get_state("c128")) * dv
        got = s.inner(p)
        assert abs(got - w) <= 1e-12 * max(1.0, abs(w)), (dt, got, w)
    # autocorrelation of the stored state with itself: (sum |psi|^2 dV)^2
    s.store_reference()
    o = s.observables(S.OBS_NORM | (1 << 11))
    assert o["autocorrelation"] == pytest.approx(o["norm"] ** 4, rel=1e-12)
    s.close()


# Precision-changing transfers convert on the device in runs of 2^22 points:
# grids of one run, of several with a ragged last one, padded and not.
@pytest.mark.parametrize("precision,n", [("c64", [64, 32, 16]), ("c128", [32, 64, 8]), ("c64", [256, 128, 256]),
                                         ("c64", [192, 128, 256]), ("c128", [256, 128, 160]), ("c64x", [96, 64, 48])])
def test_transfers_across_precisions(S, W, precision, n):
    prob = problem(W, precision, n)
    s = S.from_problem(prob)
    rng = np.random.default_rng(sum(n))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    s.set_state(x)
    stored = x.astype(np.complex64) if precision != "c128" else x
    # the state as stored, read back in both precisions
    assert np.array_equal(s.get_state("c128"), stored.astype(np.complex128))
    assert np.array_equal(s.get_state("c64"), stored.astype(np.complex64))
    # after steps: the converted read is the exact widening or rounding of
    # the read in the stored precision
    s.propagate(2)
    same = s.get_state("c128" if precision == "c128" else "c64")
    other = s.get_state("c64" if precision == "c128" else "c128")
    s.close()
    if precision == "c128":
        assert np.array_equal(other, same.astype(np.complex64))
    else:
        assert np.array_equal(other, same.astype(np.complex128))
