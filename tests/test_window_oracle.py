"""The windowed oracle reproduces the full-grid oracle at the window centre
(bitwise: same operations on the same values)."""
import numpy as np

import oracle
from paper_2207_08716_amd import inputs
from window_oracle import CELL_FIELDS, FACE_FIELDS, sample_points, window_values


def test_window_equals_full_grid():
    n, m = 36, 3
    cfg = inputs.config_mixed(n)
    f = inputs.initial_fields(cfg)
    full = oracle.Oracle(cfg.phys, n, n, n, f["phi"], f["k0"])
    full.begin_step()
    full.iterate(m)
    rng = np.random.default_rng(0)
    for p in sample_points(n, rng, 14):
        w = window_values(cfg, f["phi"], f["k0"], p, 2 * m + 4, m)
        for name in CELL_FIELDS + FACE_FIELDS:
            assert w[name] == full.f[name][p], (p, name, w[name], full.f[name][p])
