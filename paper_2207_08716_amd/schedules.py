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


def picard_step(g: Grid, n_picard: int, rtol: float, step_index: int, max_iter=1_000_000, mixed=False,
                eta_in=1e-4):
    """One physical step of the Picard schedule (pt_picard_step): per stage, a
    refresh without relaxation, a linear solve to rtol (FP64 PT sweeps, or
    FP32 sweeps inside FP64 defect correction), then the porosity time step."""
    return g.picard_step(step_index >= 1, n_picard, rtol, max_iter, mixed, eta_in)
