"""Mixed precision (FP32 correction sweeps inside FP64 defect correction)
against FP64 on the GPU and against the FP64 oracle.

The converged fields of a Picard stage must agree with the FP64 result to
relative 1e-5 per field (infinity norms)."""
import numpy as np
import pytest

import oracle
from paper_2207_08716_amd import inputs

pytestmark = pytest.mark.gpu

FIELDS = ("vx", "vy", "vz", "pt", "pf")


def _rel(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / s if s > 0 else np.abs(a - b).max()


def _grid(cfg, f):
    from paper_2207_08716_amd import schedules
    return schedules.make_grid(cfg, f)


def test_residual_matches_oracle():
    cfg = inputs.config_fp64_picard(20)
    f = inputs.initial_fields(cfg)
    g = _grid(cfg, f)
    o = oracle.Oracle(cfg.phys, 20, 20, 20, f["phi"], f["k0"])
    g.begin_step(False)
    g.iterate(45)
    o.begin_step()
    o.iterate(45)
    # one more (relaxed) refresh on both, then residuals with the same coefficients
    o.refresh()
    g.refresh()
    nm = g.residual()
    ref = o.residual()
    got = g.residual_fields()
    for a, b, name in zip(got, ref, ("fx", "fy", "fz", "rpt", "rpf")):
        assert np.abs(a - b).max() <= 1e-6 * np.abs(b).max(), name
    fmax = max(np.abs(r).max() for r in ref[:3])
    assert abs(nm["f"] - fmax) <= 1e-9 * fmax
    assert abs(nm["rpt"] - np.abs(ref[3]).max()) <= 1e-9 * np.abs(ref[3]).max()
    assert abs(nm["rpf"] - np.abs(ref[4]).max()) <= 1e-9 * np.abs(ref[4]).max()


def test_mixed_stage_matches_fp64_and_oracle():
    n = 24
    cfg = inputs.config_mixed(n)
    f = inputs.initial_fields(cfg)
    g64 = _grid(cfg, f)
    g64.begin_step(False)
    g64.refresh(1.0, 1.0)
    it64, rho64, ok64 = g64.solve_linear(1e-10, 200000)
    gmx = _grid(cfg, f)
    gmx.begin_step(False)
    gmx.refresh(1.0, 1.0)
    inner, outer, rhomx, okmx = gmx.solve_mixed(1e-10, 1e-4)
    o = oracle.Oracle(cfg.phys, n, n, n, f["phi"], f["k0"])
    o.begin_step()
    o.refresh(1.0, 1.0)
    ito, rhoo = o.solve_linear(1e-10, 200000)
    print("fp64", it64, rho64, "mixed", inner, outer, rhomx, "oracle", ito, rhoo, flush=True)
    assert ok64 and okmx and rhoo <= 1e-10
    assert outer >= 2
    for name in FIELDS:
        a, b, c = gmx.get(name), g64.get(name), o.f[name]
        assert _rel(a, b) <= 1e-5, (name, _rel(a, b))
        assert _rel(a, c) <= 1e-5, (name, _rel(a, c))
        assert _rel(b, c) <= 1e-7, (name, _rel(b, c))


def test_mixed_picard_step_matches_oracle():
    n = 16
    cfg = inputs.config_mixed(n)
    f = inputs.initial_fields(cfg)
    g = _grid(cfg, f)
    sweeps, rho, ok = g.picard_step(False, 2, 1e-10, mixed=True, eta_in=1e-4)   # pt_picard_step
    print("mixed Picard step", sweeps, rho, ok)
    assert ok
    o = oracle.Oracle(cfg.phys, n, n, n, f["phi"], f["k0"])
    counts = o.picard_step(2, 1e-10, 200000)
    print(counts)
    for name in FIELDS + ("lp", "kc", "eta", "mus"):
        r = _rel(g.get(name), o.f[name])
        assert r <= 1e-5, (name, r)


def _fp32_tall_tiles(nx, ny, nz):
    """Whether the launch cost model of the library puts the FP32 correction
    sweep on its 14-row tiles (rather than 10-row ones) for this grid: the
    best z chunk's rounds of 256 blocks times (chunk + 2) times the rows."""
    def cost(by):
        tiles = ((nx + 63) // 64) * ((ny + by - 3) // (by - 2))
        best, kz = None, 256
        while kz >= 4:
            blocks = tiles * ((nz + kz - 1) // kz)
            c = ((blocks + 255) // 256) * (min(kz, nz) + 2)
            best = c if best is None or c < best else best
            kz //= 2
        return best * by
    return cost(14) < cost(10)


def test_mixed_stage_on_tall_fp32_tiles():
    """192x84x32: the only kind of grid in these tests where the FP32
    correction sweep runs 14-row tiles (the small grids all take 10-row
    ones).  A converged mixed stage matches the FP64 stage, itself checked
    against the oracle elsewhere, within 1e-5 per field."""
    import dataclasses
    nx, ny, nz = 192, 84, 32
    assert _fp32_tall_tiles(nx, ny, nz) and not _fp32_tall_tiles(24, 24, 24)
    cfg = inputs.config_mixed(8)
    cfg = dataclasses.replace(cfg, nx=nx, ny=ny, nz=nz, name="tall-fp32")
    cfg.phys = cfg.phys.replace(lx=nx / 64, ly=ny / 64, lz=nz / 64)
    f = inputs.initial_fields(cfg)
    g64 = _grid(cfg, f)
    g64.begin_step(False)
    g64.refresh(1.0, 1.0)
    it64, rho64, ok64 = g64.solve_linear(1e-10, 400000)
    gmx = _grid(cfg, f)
    gmx.begin_step(False)
    gmx.refresh(1.0, 1.0)
    inner, outer, rhomx, okmx = gmx.solve_mixed(1e-10, 1e-4, 400000, 60)
    print("fp64", it64, rho64, "mixed", inner, outer, rhomx, flush=True)
    assert ok64 and okmx and outer >= 2
    worst = {name: _rel(gmx.get(name), g64.get(name)) for name in FIELDS}
    print(worst, flush=True)
    assert max(worst.values()) <= 1e-5, worst


def test_forced_tall_fp32_tiles_match_the_oracle_and_the_model_tiling():
    """PT_F_FP32_TALL puts the FP32 correction sweep on its 14-row tiles (the
    tiling of the 511^3 runs) on a grid where the cost model picks 10 rows:
    the mixed stage there is bitwise the stage on the model's tiling, and
    within 1e-5 of the oracle's converged stage (ragged tiles: 30 = 2 x 12 + 6
    rows, 40 columns in a 64-column tile)."""
    nx, ny, nz = 40, 30, 22
    assert not _fp32_tall_tiles(nx, ny, nz)
    cfg = inputs.config_mixed(8)
    import dataclasses
    cfg = dataclasses.replace(cfg, nx=nx, ny=ny, nz=nz, name="forced-tall")
    cfg.phys = cfg.phys.replace(lx=nx / 32, ly=ny / 32, lz=nz / 32)
    f = inputs.initial_fields(cfg)
    runs = {}
    for tall in (False, True):
        c = dataclasses.replace(cfg, phys=cfg.phys.replace(fp32_tall=tall))
        g = _grid(c, f)
        g.begin_step(False)
        g.refresh(1.0, 1.0)
        inner, outer, rho, ok = g.solve_mixed(1e-10, 1e-4, 400000, 60)
        assert ok and outer >= 2
        runs[tall] = (inner, outer, {name: g.get(name) for name in FIELDS})
    assert runs[True][:2] == runs[False][:2]
    for name in FIELDS:
        assert np.array_equal(runs[True][2][name], runs[False][2][name]), name
    o = oracle.Oracle(cfg.phys, nx, ny, nz, f["phi"], f["k0"])
    o.begin_step()
    o.refresh(1.0, 1.0)
    _ito, rhoo = o.solve_linear(1e-10, 400000)
    assert rhoo <= 1e-10
    worst = {name: _rel(runs[True][2][name], o.f[name]) for name in FIELDS}
    print(worst, flush=True)
    assert max(worst.values()) <= 1e-5, worst
