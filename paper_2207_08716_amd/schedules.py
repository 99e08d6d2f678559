"""Solve schedules built from the C entry points (host loops only)."""
from __future__ import annotations

import numpy as np

from .grid import Grid


def make_grid(cfg, fields, device="cuda") -> Grid:
    """Grid for a workload with its initial state loaded."""
    g = Grid(cfg.phys, cfg.nx, cfg.ny, cfg.nz, k0field=fields["k0"] is not None, device=device)
    g.load_initial(fields["phi"], fields["k0"])
    return g


def thesis_step(g: Grid, n_iter: int, step_index: int):
    """One physical step of the thesis schedule with a fixed iteration count."""
    g.begin_step(update_history=step_index >= 1)
    g.iterate(n_iter)


def picard_step(g: Grid, n_picard: int, rtol: float, step_index: int, max_iter=1_000_000):
    """One physical step of the Picard schedule: per stage, a refresh without
    relaxation, a linear PT solve to rtol, then the porosity time step."""
    g.begin_step(update_history=step_index >= 1)
    out = []
    for _ in range(n_picard):
        g.refresh(1.0, 1.0)
        it, rho, ok = g.solve_linear(rtol, max_iter)
        out.append((it, rho, ok))
        g.porosity_step()
    return out


def phi(g: Grid) -> np.ndarray:
    return 1.0 - np.exp(g.get("lp"))
