"""Effective memory throughput (thesis article 1, section 2.3.2).

A_eff = 2 D_unknown + D_known (eq (28)) is the minimal main-memory traffic of
one iteration: every unknown degree of freedom read and written once, every
known one read once.  T_eff = A_eff / t_it (eq (29)).  For the two-phase
solver, 12 unknown fields (three velocities, six stresses, two pressures,
porosity) and 1 known field give A_eff = (2*12 + 1) N p (eqs (35)-(38)),
N the number of grid cells and p the bytes per number.
"""
from __future__ import annotations

N_UNKNOWN = 12
N_KNOWN = 1


def a_eff_bytes(n_cells: int, p_bytes: int, n_unknown: int = N_UNKNOWN,
                n_known: int = N_KNOWN) -> float:
    """Minimal bytes per iteration, eq (37) without the 1e-9 factor."""
    return float((2 * n_unknown + n_known) * n_cells * p_bytes)


def t_eff_gbs(n_cells: int, p_bytes: int, t_it_s: float, n_unknown: int = N_UNKNOWN,
              n_known: int = N_KNOWN) -> float:
    """T_eff in GB/s (1 GB = 1e9 bytes), eq (38)."""
    return a_eff_bytes(n_cells, p_bytes, n_unknown, n_known) * 1e-9 / t_it_s


def parallel_efficiency(t_seq: float, t_par: float, n_proc: int) -> float:
    """E(N, P) = T_seq / (P T(N, P)), eq (31)."""
    return t_seq / (n_proc * t_par)


def overhead_share(overhead: float, speedup: float) -> float:
    """Share of a fixed parallel overhead once the computation is `speedup`
    times faster: o / (o + (1 - o)/speedup) (footnote 3 of article 1)."""
    return overhead / (overhead + (1.0 - overhead) / speedup)
