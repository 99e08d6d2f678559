"""Oracle values at single points of a large grid, computed on a window.

After m PT iterations from the seeded initial state a value depends only on
the initial fields within a few cells (each iteration reaches at most two
cells further: velocities through the stresses, pressures through the
divergence and the Darcy flux).  Running the oracle on a window of half-width
r > 2m + 2 around a point therefore reproduces the full-grid value there;
window sides that fall on the domain boundary carry the true boundary
conditions, the others are far enough away.  The spacing, the damping and
the Pt pseudo-step are the full grid's.
"""
import numpy as np

import oracle

CELL_FIELDS = ("pt", "pf", "lp")
FACE_FIELDS = ("vx", "vy", "vz", "rx", "ry", "rz")


def window_values(cfg, phi, k0, point, r, n_iter):
    """Oracle values of the cell fields and the low faces of cell `point`
    (k, j, i) after the thesis schedule's refresh + n_iter iterations."""
    k, j, i = point
    lo = [max(0, c - r) for c in (k, j, i)]
    hi = [min(n, c + r + 1) for c, n in zip((k, j, i), (cfg.nz, cfg.ny, cfg.nx))]
    sl = tuple(slice(a, b) for a, b in zip(lo, hi))
    wz, wy, wx = (b - a for a, b in zip(lo, hi))
    ph = cfg.phys
    o = oracle.Oracle(ph, wx, wy, wz, np.ascontiguousarray(phi[sl]),
                      None if k0 is None else np.ascontiguousarray(k0[sl]),
                      global_counts=(cfg.nx, cfg.ny, cfg.nz))
    o.begin_step()
    o.iterate(n_iter)
    lk, lj, li = k - lo[0], j - lo[1], i - lo[2]
    out = {name: o.f[name][lk, lj, li] for name in CELL_FIELDS + FACE_FIELDS}
    return out


def sample_points(n, rng, count):
    """Corners, tile and z-chunk seams and random interior cells."""
    pts = set()
    for k in (0, n - 1):
        for j in (0, n - 1):
            for i in (0, n - 1):
                pts.add((k, j, i))
    seams = [c for c in (1, 5, 6, 7, 61, 62, 63, 64, 123, 124, 127, 128, n // 2, n - 2) if 0 <= c < n]
    while len(pts) < count:
        if rng.random() < 0.5:
            pts.add(tuple(int(rng.choice(seams)) for _ in range(3)))
        else:
            pts.add(tuple(int(v) for v in rng.integers(0, n, 3)))
    return sorted(pts)
