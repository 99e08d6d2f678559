"""Parity at the sizes of the FP64-Picard and mixed workloads: the 255^3
Picard workload under the thesis schedule against the oracle on the full
grid; a converged Picard step against the oracle; a mixed-precision Picard
step against the FP64 one at 127^3."""
import time

import numpy as np
import pytest

import oracle
from paper_2207_08716_amd import inputs

from test_gpu_parity import COEF, STATE, _compare, _pair, _rel

pytestmark = pytest.mark.gpu


def test_fp64_picard_workload_255_thesis_iterations():
    # the 255^3 workload (lognormal k0) in its launch configuration, 200
    # iterations of the thesis schedule (14 refreshes, 13 norm checks), every
    # field compared over the whole grid
    cfg = inputs.config_fp64_picard(255)
    print("255^3 thesis-schedule parity: set-up", flush=True)
    g, o = _pair(cfg)
    g.begin_step(False)
    g.iterate(200)
    t0 = time.time()
    o.begin_step()
    done = 0
    while done < 200:
        k = min(20, 200 - done)
        o.iterate(k)
        done += k
        print(f"oracle 255^3: {done} iterations, {time.time() - t0:.0f} s", flush=True)
    _compare(g, o, STATE + COEF)


def test_picard_step_converged_matches_oracle():
    # one physical step of 5 Picard stages, every linear solve to 1e-9: the
    # converged fields agree to the solve tolerance
    n, rtol = 32, 1e-9
    cfg = inputs.config_fp64_picard(n)
    g, o = _pair(cfg)
    sweeps, rho, ok = g.picard_step(False, 5, rtol)        # the library's Picard driver
    assert ok
    o.begin_step()
    its = []
    for p in range(5):
        o.refresh(1.0, 1.0)
        it_o, rho_o = o.solve_linear(rtol, 2_000_000)
        assert rho_o <= rtol
        its.append(it_o)
        o.porosity_step()
    print(f"GPU {sweeps} sweeps rho {rho:.2e}; oracle {sum(its)} iterations {its}", flush=True)
    assert sweeps == sum(its)
    worst = {k: _rel(g.get(k), o.f[k]) for k in ("vx", "vy", "vz", "pt", "pf", "lp")}
    print(worst, flush=True)
    assert max(worst.values()) <= 1e-7, worst


def test_mixed_picard_step_matches_fp64_127():
    # the mixed workload at 127^3, one Picard step of 5 stages to 1e-8: FP32
    # sweeps inside FP64 defect correction against FP64 PT sweeps
    from paper_2207_08716_amd import schedules
    n, rtol = 127, 1e-8
    cfg = inputs.config_mixed(n)
    f = inputs.initial_fields(cfg)
    out = {}
    for mode in ("fp64", "mixed"):
        g = schedules.make_grid(cfg, f)
        if mode == "mixed":
            g.enable_mixed()
        g.begin_step(False)
        t0 = time.time()
        for p in range(5):
            g.refresh(1.0, 1.0)
            if mode == "fp64":
                it, rho, ok = g.solve_linear(rtol, 2_000_000)
            else:
                inner, outer, rho, ok = g.solve_mixed(rtol, 1e-4, 2_000_000, 60)
            print(f"{mode} stage {p}: rho {rho:.2e} ({time.time() - t0:.1f} s)", flush=True)
            assert ok
            g.porosity_step()
        out[mode] = {k: g.get(k) for k in ("vx", "vy", "vz", "pt", "pf", "lp")}
        g.close()
    worst = {k: _rel(out["mixed"][k], out["fp64"][k]) for k in out["fp64"]}
    print(worst, flush=True)
    assert max(worst.values()) <= 1e-5, worst


def _flips_and_yield(g, ph):
    """Cells at the decompaction switch (|Pf - Pt| below 1e-12 of the largest
    pressure) and the fraction of cells whose viscosity the cap cut."""
    pt, pf, mn = g.get("pt"), g.get("pf"), g.get("mn")
    scale = max(np.abs(pt).max(), np.abs(pf).max(), 1e-300)
    flips = int((np.abs(pf - pt) < 1e-12 * scale).sum())
    return flips, float((mn < ph.mu0 * (1 - 1e-12)).mean())


def test_mixed_workload_with_an_engaging_cap_matches_oracle():
    """The mixed workload's recipe with a cohesion small enough for the cap to
    engage (C = 4e-3, floor 2e-3: about 12 % of the cells yield; with C = 1
    the stresses stay far below the yield stress, and below C ~ 1e-3 the
    viscosity contrast makes the PT iteration diverge): a converged FP64
    Picard step (5 stages to 1e-9) and the mixed one against the oracle's."""
    n, rtol = 24, 1e-9
    cfg = inputs.config_mixed(n)
    cfg.phys = cfg.phys.replace(coh=4e-3, tau_y_min=2e-3)
    g, o = _pair(cfg)
    sweeps, rho, ok = g.picard_step(False, 5, rtol)
    assert ok
    counts = o.picard_step(5, rtol, 2_000_000)
    flips, yielded = _flips_and_yield(g, cfg.phys)
    print(f"GPU {sweeps} sweeps; oracle {[c[0] for c in counts]}; flips {flips}, yielded {yielded:.3f}",
          flush=True)
    assert yielded > 0.05
    assert sweeps == sum(c[0] for c in counts)
    worst = {k: _rel(g.get(k), o.f[k]) for k in ("vx", "vy", "vz", "pt", "pf", "lp", "mn")}
    print(worst, flush=True)
    assert max(worst.values()) <= 1e-7, worst
    from paper_2207_08716_amd import schedules
    f = inputs.initial_fields(cfg)
    m = schedules.make_grid(cfg, f)
    _s, _r, okm = m.picard_step(False, 5, rtol, mixed=True)
    assert okm
    worst = {k: _rel(m.get(k), o.f[k]) for k in ("vx", "vy", "vz", "pt", "pf", "lp")}
    print("mixed", worst, flush=True)
    assert max(worst.values()) <= 1e-5, worst
