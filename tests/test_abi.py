"""The C-ABI library loads and exports every entry point the header declares;
argument validation happens on the host before any launch (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2207_08716_amd import abi, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="ptporo.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(abi.LIB_PATH):
        pytest.skip("libptporo.so not built")
    return abi.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "pt_iteration" in names and "pt_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abi.EXPORTS)


def test_every_waves_symbol_is_exported(lib):
    names = _declared("ptwaves.h")
    assert "pt_waves_iterate" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abi.WAVES_EXPORTS)


def test_waves_entry_points_validate_on_the_host(lib):
    ph = inputs.WavePhysics()
    p = abi.waves_params_from(ph)
    h = C.c_void_p()
    assert lib.pt_waves_create(1, 4, 4, 32, C.byref(p), C.byref(h)) == -1
    assert lib.pt_waves_create(4, 4, 4, 4, C.byref(p), C.byref(h)) == -1     # pitch < nx + 1
    for bad in (dict(dt=0.0), dict(tau=-1.0), dict(phi_min=0.0), dict(phi_max=1.5), dict(xs_max=1.0),
                dict(c_pf=float("nan")), dict(nup=0)):
        q = abi.waves_params_from(ph.replace(**bad))
        assert lib.pt_waves_create(4, 4, 4, 32, C.byref(q), C.byref(h)) == -1, bad
    q = abi.waves_params_from(ph)
    q.version = 7
    assert lib.pt_waves_create(4, 4, 4, 32, C.byref(q), C.byref(h)) == -1
    assert lib.pt_waves_create(4, 5, 6, 32, C.byref(p), C.byref(h)) == 0
    try:
        assert lib.pt_waves_field_elems(h) == 7 * 6 * 32
        assert lib.pt_waves_bind_field(h, 0, 0, C.c_void_p(0x1008)) == -1
        assert lib.pt_waves_bind_field(h, 9, 0, C.c_void_p(0x1000)) == -1
        assert lib.pt_waves_bind_field(h, abi.WAVES_FIELD_ID["pf_old"], 1, C.c_void_p(0x1000)) == -1
        assert b"copy" in lib.pt_waves_last_message(h)
        # nothing bound: every launching call refuses before touching the device
        assert lib.pt_waves_begin_step(h) == -1
        assert lib.pt_waves_iterate(h, 1) == -1
        assert b"bound" in lib.pt_waves_last_message(h)
        it, e = C.c_int64(), C.c_double()
        assert lib.pt_waves_solve_step(h, 1e-8, 100, C.byref(it), C.byref(e)) == -1
        assert lib.pt_waves_solve_step(h, 0.0, 100, C.byref(it), C.byref(e)) == -1
        assert lib.pt_waves_last_error(h, C.byref(e)) == -1              # nothing computed yet
        sz = C.c_size_t()
        assert lib.pt_waves_workspace_size(h, C.byref(sz)) == 0 and sz.value > 0
        assert lib.pt_waves_bind_workspace(h, C.c_void_p(0x1000), 8) == -1
        cp = C.c_int32()
        assert lib.pt_waves_current(h, abi.WAVES_FIELD_ID["pf"], C.byref(cp)) == 0 and cp.value == 0
    finally:
        lib.pt_waves_destroy(h)


def test_create_validates_arguments(lib):
    p = abi.params_from(inputs.Physics(), False)
    h = C.c_void_p()
    assert lib.pt_create(1, 4, 4, 8, C.byref(p), C.byref(h)) == -1
    assert lib.pt_create(4, 4, 4, 4, C.byref(p), C.byref(h)) == -1   # pitch < nx + 1
    bad = abi.params_from(inputs.Physics(dt=0.0), False)
    assert lib.pt_create(4, 4, 4, 8, C.byref(bad), C.byref(h)) == -1
    bad = abi.params_from(inputs.Physics(), False)
    bad.version = 99
    assert lib.pt_create(4, 4, 4, 8, C.byref(bad), C.byref(h)) == -1
    assert lib.pt_create(4, 5, 6, 8, C.byref(p), C.byref(h)) == 0
    try:
        assert lib.pt_field_elems(h) == 7 * 6 * 8
        # unaligned, null, bad id, bad copy
        assert lib.pt_bind_field(h, 0, 0, C.c_void_p(0x1008)) == -1
        assert lib.pt_bind_field(h, 0, 0, None) == -1
        assert lib.pt_bind_field(h, 99, 0, C.c_void_p(0x1000)) == -1
        assert lib.pt_bind_field(h, abi.FIELD_ID["mus"], 1, C.c_void_p(0x1000)) == -1
        assert b"copy" in lib.pt_last_error(h)
        # nothing bound: every launching call refuses before touching the device
        assert lib.pt_iteration(h, 1, 0) == -1
        assert lib.pt_begin_step(h, 0) == -1
        assert lib.pt_refresh(h, 0.5, 0.5) == -1
        sz = C.c_size_t()
        assert lib.pt_workspace_size(h, C.byref(sz)) == 0 and sz.value > 0
        assert lib.pt_bind_workspace(h, C.c_void_p(0x1000), 8) == -1
    finally:
        lib.pt_destroy(h)
    assert lib.pt_status_str(-3) == b"diverged (non-finite norm)"


def test_driver_and_adjoint_entry_points_validate_on_the_host(lib):
    p = abi.params_from(inputs.Physics(), True)
    h = C.c_void_p()
    assert lib.pt_create(6, 5, 4, 32, C.byref(p), C.byref(h)) == 0
    try:
        box = lib.pt_field_elems(h) * 8
        sweeps, rho = C.c_int64(), C.c_double()
        # argument checks
        assert lib.pt_picard_step(h, 0, 0, 1e-8, 100, 0, 1e-4, C.byref(sweeps), C.byref(rho)) == -1
        assert lib.pt_picard_step(h, 0, 2, 0.0, 100, 0, 1e-4, C.byref(sweeps), C.byref(rho)) == -1
        assert lib.pt_picard_step(h, 0, 2, 1e-8, 100, 1, 1.5, C.byref(sweeps), C.byref(rho)) == -1
        # nothing bound: refused before any launch
        assert lib.pt_picard_step(h, 0, 2, 1e-8, 100, 0, 1e-4, C.byref(sweeps), C.byref(rho)) == -1
        inner, outer = C.c_int64(), C.c_int32()
        assert lib.pt_solve_mixed(h, 1e-8, 1e-4, 10, 2, C.byref(inner), C.byref(outer), C.byref(rho)) == -1
        assert lib.pt_solve_linear(h, 1e-8, 10, C.byref(inner), C.byref(rho)) == -1
        # workspaces: sizes and binding checks
        sz = C.c_size_t()
        elems = lib.pt_field_elems(h)
        assert lib.pt_mixed_workspace_size(h, C.byref(sz)) == 0 and sz.value == 24 * (elems + 64) * 4
        assert lib.pt_bind_mixed_workspace(h, C.c_void_p(0x1008), sz.value) == -1
        assert lib.pt_adjoint_workspace_size(h, 0, C.byref(sz)) == -1
        assert lib.pt_adjoint_workspace_size(h, 16, C.byref(sz)) == 0 and sz.value >= 40 * box
        # tape sizes: every stage (8 boxes), or step checkpoints (15) + one step's stages
        assert lib.pt_adjoint_tape_size(h, 3, 5, 0, C.byref(sz)) == 0 and sz.value == 3 * 5 * 8 * box
        assert lib.pt_adjoint_tape_size(h, 3, 5, abi.ADJ_CHECKPOINT, C.byref(sz)) == 0
        assert sz.value == (3 * 15 + 5 * 8) * box
        assert lib.pt_adjoint_tape_size(h, 0, 5, 0, C.byref(sz)) == -1
        J, fit, ait = C.c_double(), C.c_int64(), C.c_int64()
        sensors = (C.c_int64 * 2)(1, 2)
        d_obs = (C.c_double * 2)(0.0, 0.0)
        assert lib.pt_adjoint_run(h, 1, 1, 0, 1e-8, 1e-8, 100, None, 2, d_obs, C.c_void_p(0x1000), 1 << 20,
                                  C.c_void_p(0x1000), C.byref(J), C.byref(fit), C.byref(ait)) == -1
        assert lib.pt_adjoint_run(h, 1, 1, 0, 1e-8, 1e-8, 100, sensors, 2, d_obs, C.c_void_p(0x1000), 1 << 20,
                                  C.c_void_p(0x1000), C.byref(J), C.byref(fit), C.byref(ait)) == -1
        assert lib.pt_set_progress(h, abi.PROGRESS_FN(), None) == 0
        # state set-up refuses an unbound grid
        assert lib.pt_reset_state(h) == -1
        assert lib.pt_set_porosity(h, C.c_void_p(0x1000)) == -1
        assert lib.pt_set_porosity(h, C.c_void_p(0x1008)) == -1
    finally:
        lib.pt_destroy(h)


def test_multigrid_entry_points_validate_on_the_host(lib):
    p = abi.params_from(inputs.Physics(), False)
    h = C.c_void_p()
    assert lib.pt_create(63, 40, 17, 64, C.byref(p), C.byref(h)) == 0
    try:
        sz = C.c_size_t()
        good = abi.mg_params()
        assert lib.pt_mg_workspace_size(h, C.byref(good), C.byref(sz)) == 0 and sz.value > 0
        # 63 x 40 x 17 -> 32 x 20 x 9 -> 16 x 10 x 5: the automatic hierarchy
        # stops at the first grid with an axis of at most 8 cells
        three = abi.mg_params(levels=3)
        sz3 = C.c_size_t()
        assert lib.pt_mg_workspace_size(h, C.byref(three), C.byref(sz3)) == 0 and sz3.value == sz.value
        # a fourth grid (8 x 5 x 3) is allowed on request; a fifth would halve
        # an axis of 3 cells
        assert lib.pt_mg_workspace_size(h, C.byref(abi.mg_params(levels=4)), C.byref(sz)) == 0
        assert lib.pt_mg_workspace_size(h, C.byref(abi.mg_params(levels=5)), C.byref(sz)) == -1
        for bad in (dict(levels=1), dict(levels=13), dict(nu1=0), dict(nu2=-1), dict(coarse_sweeps=0),
                    dict(n_pt=0), dict(c_v=0.0), dict(c_pf=float("nan")), dict(krylov=-1),
                    dict(krylov=abi.MG_MAX_KRYLOV + 1), dict(eta_mean=3)):
            q = abi.mg_params(**bad)
            assert lib.pt_mg_workspace_size(h, C.byref(q), C.byref(sz)) == -1, bad
        q = abi.mg_params()
        q.version = 1
        assert lib.pt_mg_workspace_size(h, C.byref(q), C.byref(sz)) == -1
        for bad in (-1, 3):
            assert lib.pt_mg_workspace_size(h, C.byref(abi.mg_params(eta_mean=bad)), C.byref(sz)) == -1
        # Krylov acceleration: 5 (m + 1) FP64 and 5 (m + 1) FP32 fine boxes more
        # (plus the skews between boxes and the partial sums of the inner products)
        box = 64 * 41 * 18
        for m in (1, abi.MG_MAX_KRYLOV):
            szk = C.c_size_t()
            assert lib.pt_mg_workspace_size(h, C.byref(abi.mg_params(krylov=m)), C.byref(szk)) == 0
            extra = szk.value - sz3.value
            need = 5 * (m + 1) * box * 8 + 5 * (m + 1) * box * 4
            assert need <= extra <= need + (1 << 20), (m, extra, need)
        assert lib.pt_bind_mg_workspace(h, C.byref(good), C.c_void_p(0x1008), 1 << 40) == -1
    finally:
        lib.pt_destroy(h)
    # the Krylov kernels move 4 columns as one vector: a pitch of 41 is refused
    h = C.c_void_p()
    assert lib.pt_create(40, 31, 31, 41, C.byref(p), C.byref(h)) == 0
    try:
        k8 = abi.mg_params(krylov=8)
        assert lib.pt_mg_workspace_size(h, C.byref(k8), C.byref(sz)) == 0
        assert lib.pt_bind_mg_workspace(h, C.byref(k8), C.c_void_p(0x1000), 1 << 40) == -1
        assert b"multiple of 4" in lib.pt_last_error(h)
    finally:
        lib.pt_destroy(h)
    h = C.c_void_p()
    assert lib.pt_create(63, 40, 17, 64, C.byref(p), C.byref(h)) == 0
    try:
        assert lib.pt_bind_mg_workspace(h, C.byref(good), C.c_void_p(0x1000), 8) == -1
        n = C.c_int32()
        assert lib.pt_mg_levels(h, C.byref(n), None) == 0 and n.value == 0
        cyc, rho = C.c_int64(), C.c_double()
        assert lib.pt_solve_mg(h, 0.0, 10, C.byref(cyc), C.byref(rho)) == -1
        assert lib.pt_solve_mg(h, 1e-8, -1, C.byref(cyc), C.byref(rho)) == -1
        assert lib.pt_solve_mg(h, 1e-8, 10, C.byref(cyc), C.byref(rho)) == -1      # nothing bound
        assert lib.pt_picard_step(h, 0, 2, 1e-8, 100, abi.SOLVER_MG, 0.0, C.byref(cyc), C.byref(rho)) == -1
        assert b"multigrid" in lib.pt_last_error(h)
        assert lib.pt_picard_step(h, 0, 2, 1e-8, 100, 3, 0.0, C.byref(cyc), C.byref(rho)) == -1
    finally:
        lib.pt_destroy(h)


def test_counters_round_trip_on_the_host(lib):
    """pt_get_counters / pt_set_counters carry the host-side state of a handle
    to another one (no device call)."""
    p = abi.params_from(inputs.Physics(), False)
    h1, h2 = C.c_void_p(), C.c_void_p()
    assert lib.pt_create(6, 5, 4, 32, C.byref(p), C.byref(h1)) == 0
    assert lib.pt_create(6, 5, 4, 32, C.byref(p), C.byref(h2)) == 0
    try:
        c = abi.Counters()
        assert lib.pt_get_counters(h1, C.byref(c)) == 0
        assert c.version == abi.ABI_VERSION and c.iter == 0 and c.ref_set == 0 and list(c.cur) == [0] * abi.NPING
        # a new handle: R is in its fields, V's other copy holds no iterate
        assert (c.r_stored, c.v_prev) == (1, 0)
        c.iter, c.refreshed, c.ref_set, c.ref_v, c.ref_p = 37, 1, 1, 2.5, 0.125
        c.r_stored, c.v_prev = 0, 1
        c.cur[0], c.cur[5], c.mixed_copy = 1, 1, 1
        assert lib.pt_set_counters(h2, C.byref(c)) == 0
        d = abi.Counters()
        assert lib.pt_get_counters(h2, C.byref(d)) == 0
        assert (d.iter, d.refreshed, d.ref_set, d.ref_v, d.ref_p) == (37, 1, 1, 2.5, 0.125)
        assert list(d.cur) == [1, 0, 0, 0, 0, 1, 0, 0, 0] and d.mixed_copy == 1
        assert d.mixed_clean == 0                       # no mixed workspace bound
        assert (d.r_stored, d.v_prev) == (0, 1)
        gv, gp = C.c_double(), C.c_double()
        assert lib.pt_residual_reference(h2, C.byref(gv), C.byref(gp)) == 0 and (gv.value, gp.value) == (2.5, 0.125)
        cur = C.c_int32()
        assert lib.pt_current(h2, 5, C.byref(cur)) == 0 and cur.value == 1
        for field, value in (("version", 99), ("iter", -1), ("mixed_copy", 2), ("r_stored", 2), ("v_prev", 0)):
            bad = abi.Counters()
            C.memmove(C.byref(bad), C.byref(c), C.sizeof(c))
            setattr(bad, field, value)
            assert lib.pt_set_counters(h2, C.byref(bad)) == -1, field
        bad = abi.Counters()
        C.memmove(C.byref(bad), C.byref(c), C.sizeof(c))
        bad.cur[3] = 2
        assert lib.pt_set_counters(h2, C.byref(bad)) == -1
    finally:
        lib.pt_destroy(h1)
        lib.pt_destroy(h2)
