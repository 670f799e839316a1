"""wp_propagate_observe_noalloc through the C ABI: the same results as
wp_propagate_observe, bit for bit, on calls in a row that share the
library's fixed per-device moment array (the second with a smaller grid, so
rows the first call left behind lie beyond what the second reads), and its
rejections."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MOMENTS = 0x7F | 0x700  # norm, <x_d>, <x_d^2>, widths


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


def observe(S, sim, nsteps, noalloc):
    out = (C.c_double * 12)()
    f = S.lib.wp_propagate_observe_noalloc if noalloc else S.lib.wp_propagate_observe
    rc = f(sim._h, int(nsteps), MOMENTS, out)
    assert rc == 0, (rc, S.lib.wp_last_error(sim._h).decode())
    return np.array(out[:11])


def pair(S, prob, precision, slabs=None):
    """Two handles with the same grid, potential and Gaussian state."""
    a = S.from_problem(prob, precision=precision)
    b = S.from_problem(prob, precision=precision)
    if slabs:
        a.set_slabs(slabs)
        b.set_slabs(slabs)
    return a, b


def check_same(S, prob, precision, nsteps, slabs=None):
    a, b = pair(S, prob, precision, slabs)
    want = observe(S, a, nsteps, noalloc=False)
    got = observe(S, b, nsteps, noalloc=True)
    sa, sb = a.get_state(precision if precision != "c64x" else "c64"), b.get_state(
        precision if precision != "c64x" else "c64")
    ta, tb = a.time(), b.time()
    a.close()
    b.close()
    assert np.array_equal(got, want), (got, want)
    assert np.array_equal(sa, sb)
    assert ta == tb
    return got


def test_noalloc_two_calls_in_a_row_smaller_second(S, W):
    big = W.softcore_3d(n=64, steps=0, precision="c64", half_width=5.0)
    big.t0 = 9.0
    o1 = check_same(S, big, "c64", 7)
    small = W.modulated_trap_2d(n=128, steps=0, precision="c64", half_width=8.0)
    o2 = check_same(S, small, "c64", 5)
    assert abs(o1[0] - 1.0) < 1e-5 and abs(o2[0] - 1.0) < 1e-5


@pytest.mark.parametrize("precision", ["c128", "c64x"])
def test_noalloc_other_precisions(S, W, precision):
    prob = W.softcore_3d(n=32, steps=0, precision=precision, half_width=5.0)
    prob.t0 = 9.5
    check_same(S, prob, precision, 4)
    small = W.modulated_trap_2d(n=64, steps=0, precision=precision, half_width=8.0)
    check_same(S, small, precision, 3)


def test_noalloc_slabs_on_one_stream(S, W):
    """A fresh 3D handle with several x slabs: its second stream does not
    exist yet, so the no-alloc call runs every slab on the handle's stream;
    wp_propagate_observe runs them on two.  Same bits."""
    prob = W.softcore_3d(n=64, steps=0, precision="c64", half_width=5.0)
    check_same(S, prob, "c64", 3, slabs=4)


def test_noalloc_rejections(S, W):
    # 1D grid, and a mask with the energy: not the fused case
    for prob in (W.driven_ho_1d(n=256, steps=0, precision="c64"),):
        s = S.from_problem(prob)
        out = (C.c_double * 12)()
        assert S.lib.wp_propagate_observe_noalloc(s._h, 3, MOMENTS, out) == -4  # WP_EUNSUPPORTED
        s.close()
    s = S.from_problem(W.modulated_trap_2d(n=64, steps=0, precision="c64", half_width=8.0))
    out = (C.c_double * 12)()
    assert S.lib.wp_propagate_observe_noalloc(s._h, 3, 0xFF, out) == -4
    assert S.lib.wp_propagate_observe_noalloc(s._h, 0, MOMENTS, out) == -1  # WP_EINVAL
    assert S.lib.wp_propagate_observe_noalloc(s._h, 3, MOMENTS, None) == -1
    s.close()
    # no state yet: a handle created through the C ABI with nothing bound
    prob = W.modulated_trap_2d(n=64, steps=0, precision="c64", half_width=8.0)
    g, p = S.grid_desc(prob.grid, "c64"), S.potential_desc(prob.pot)
    h = C.c_void_p()
    assert S.lib.wp_create(C.byref(g), C.byref(p), None, C.byref(h)) == 0
    assert S.lib.wp_propagate_observe_noalloc(h, 3, MOMENTS, out) == -5  # WP_ESTATE
    # more workgroups in the closing pass than the fixed array has rows: a
    # first axis of 512 points with 2^21 lines across it (16 lines per
    # workgroup); rejected before anything runs
    big = W.softcore_3d(n=4, steps=0, precision="c64")
    big.grid.n = [512, 2048, 1024]
    g2 = S.grid_desc(big.grid, "c64")
    h2 = C.c_void_p()
    assert S.lib.wp_create(C.byref(g2), C.byref(p), None, C.byref(h2)) == 0
    assert S.lib.wp_propagate_observe_noalloc(h2, 3, MOMENTS, out) == -4
    assert b"rows" in S.lib.wp_last_error(h2)
    assert S.lib.wp_destroy(h) == 0 and S.lib.wp_destroy(h2) == 0
