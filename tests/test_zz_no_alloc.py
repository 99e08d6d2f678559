"""pt_solve_linear_static, the entry point that allocates nothing: through
the C ABI it gives the same solve as pt_solve_linear, bit for bit, on two
calls in a row (the second on a smaller grid, so the static scratch holds
the first call's larger contents), and it refuses grids beyond its scratch
on the host."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2207_08716_amd import abi, inputs

STATE = ("vx", "vy", "vz", "pt", "pf", "rx", "ry", "rz")


def test_static_scratch_refuses_oversized_grids_on_the_host():
    if not os.path.exists(abi.LIB_PATH):
        pytest.skip("libptporo.so not built")
    lib = abi.load()
    p = abi.params_from(inputs.Physics(), False)
    h = C.c_void_p()
    # 1400^3 cells: 22 x 280 x 6 norm blocks, beyond the 16382 of the scratch
    assert lib.pt_create(1400, 1400, 1400, 1408, C.byref(p), C.byref(h)) == 0
    try:
        it, rho = C.c_int64(), C.c_double()
        assert lib.pt_solve_linear_static(h, 1e-8, 10, C.byref(it), C.byref(rho)) == -1
        assert b"static scratch" in lib.pt_last_error(h)
        assert lib.pt_solve_linear_static(h, 0.0, 10, C.byref(it), C.byref(rho)) == -1
    finally:
        lib.pt_destroy(h)


def _stage(cfg, static):
    from paper_2207_08716_amd import schedules
    f = inputs.initial_fields(cfg)
    g = schedules.make_grid(cfg, f)
    g.begin_step(False)
    g.refresh(1.0, 1.0)
    solve = g.solve_linear_static if static else g.solve_linear
    it, rho, ok = solve(1e-9)
    assert ok
    out = {n: g.get(n) for n in STATE}
    g.close()
    return it, rho, out


@pytest.mark.gpu
def test_static_solve_equals_the_workspace_solve_on_two_calls():
    for n in (28, 12):                       # second call: a smaller grid
        cfg = inputs.config_mixed(n)
        it_s, rho_s, f_s = _stage(cfg, static=True)
        it_w, rho_w, f_w = _stage(cfg, static=False)
        assert it_s == it_w and rho_s == rho_w, (n, it_s, it_w, rho_s, rho_w)
        for name in STATE:
            assert np.array_equal(f_s[name], f_w[name]), (n, name)
