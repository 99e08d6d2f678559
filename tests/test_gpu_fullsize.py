"""Full-size check at 511^3 in the launch configuration the benchmark times:
the GPU's refresh + 3 thesis-schedule iterations against the oracle run on
windows around sampled points (corners, tile and z-chunk seams, interior);
see window_oracle.py for why a window reproduces the full-grid value."""
import numpy as np
import pytest

from paper_2207_08716_amd import inputs
from window_oracle import CELL_FIELDS, FACE_FIELDS, sample_points, window_values

pytestmark = pytest.mark.gpu


def test_fullsize_511_sampled_against_windowed_oracle():
    import torch
    from paper_2207_08716_amd import schedules
    n, m = 511, 3
    cfg = inputs.config_mixed(n)
    f = inputs.initial_fields(cfg)
    g = schedules.make_grid(cfg, f)
    g.begin_step(False)
    g.iterate(m)
    pts = sample_points(n, np.random.default_rng(11), 48)
    kk, jj, ii = (torch.tensor([p[a] for p in pts], device="cuda") for a in range(3))
    got = {}
    with torch.cuda.stream(g.stream):
        for name in CELL_FIELDS + FACE_FIELDS:
            got[name] = g.view(name)[kk, jj, ii].cpu().numpy()
    ref = {name: np.zeros(len(pts)) for name in got}
    for q, p in enumerate(pts):
        w = window_values(cfg, f["phi"], f["k0"], p, 2 * m + 4, m)
        for name in got:
            ref[name][q] = w[name]
    worst = {}
    for name in got:
        scale = np.abs(ref[name]).max()
        worst[name] = float(np.abs(got[name] - ref[name]).max() / scale) if scale > 0 else 0.0
    print(worst, flush=True)
    assert all(v <= 1e-12 for v in worst.values()), worst
    assert np.abs(ref["vz"]).max() > 0 and np.abs(ref["pf"]).max() > 0
