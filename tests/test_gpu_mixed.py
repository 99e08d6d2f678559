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
