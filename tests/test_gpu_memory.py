"""A state too large for the device: the library refuses it with WP_ENOMEM
at its first use (the handle itself, a few KB of tables, is created), keeps
refusing calls that need it, and destroys cleanly; the failed allocation
leaves nothing behind, so the next handle on the same thread runs and its
launches report success."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu

WP_ENOMEM = -2


@pytest.fixture(scope="module")
def S():
    from paper_1306_3247_amd import sim

    return sim


@pytest.fixture(scope="module")
def W():
    from paper_1306_3247_amd import workloads

    return workloads


def test_state_larger_than_the_device(S, W):
    import torch

    # 4096^3 points in FP64: a 1 TiB state against 288 GB of HBM
    prob = W.softcore_3d(n=4096, steps=0, precision="c128", half_width=320.0)
    g, p = S.grid_desc(prob.grid, "c128"), S.potential_desc(prob.pot)
    need = C.c_uint64()
    assert S.lib.wp_state_bytes(C.byref(g), C.byref(need)) == 0
    assert need.value >= 16 * 4096 ** 3
    assert need.value > torch.cuda.get_device_properties(0).total_memory
    h = C.c_void_p()
    stream = torch.cuda.current_stream()
    assert S.lib.wp_create(C.byref(g), C.byref(p), C.c_void_p(stream.cuda_stream), C.byref(h)) == 0
    try:
        zero, one = (C.c_double * 3)(0.0, 0.0, 0.0), (C.c_double * 3)(1.0, 1.0, 1.0)
        rc = S.lib.wp_set_state_gaussian(h, zero, one, zero, 0.0)
        assert rc == WP_ENOMEM, rc
        assert b"out of device memory" in S.lib.wp_last_error(h)
        assert S.lib.wp_propagate(h, 1) == WP_ENOMEM
    finally:
        assert S.lib.wp_destroy(h) == 0

    small = W.softcore_3d(n=32, steps=0, precision="c64", half_width=5.0)
    small.t0 = 9.5
    s = S.from_problem(small)
    s.propagate(3)
    norm = s.observables(S.OBS_NORM)["norm"]
    s.close()
    assert abs(norm - 1.0) <= 1e-5
