"""Pins of the oracle's stage adjoint: against a dense transposed solve on a
tiny grid, and against central finite differences of the misfit."""
import numpy as np

import oracle
from oracle import adjoint
from paper_2207_08716_amd import inputs

from test_oracle_pins import _jacobian, _pack_state, _unpack_state, _blocks  # noqa: F401


def _stage_setup(n, seed=21):
    cfg = inputs.config_adjoint(n)
    phi = inputs.porosity_field(cfg)
    logk0 = np.log(inputs.k0_field(cfg))
    rng = np.random.default_rng(seed)
    sensors = np.sort(rng.choice(np.arange(n ** 3), size=6, replace=False))
    return cfg, phi, logk0, sensors


def test_adjoint_solution_equals_dense_transposed_solve():
    n = 4
    cfg, phi, logk0, sensors = _stage_setup(n)
    fwd = adjoint.stage_forward(cfg.phys, n, n, n, phi, logk0, 1e-13)
    d = np.zeros(len(sensors))
    J, g = adjoint.misfit(fwd.f["pf"], sensors, d)
    lam, it, rho = adjoint.solve_adjoint(fwd, g, rtol=1e-13)
    # dense: probe the stage residual Jacobian and solve J^T lam = (0, 0, g)
    x0 = _pack_state(fwd, n)
    JF, _ = _jacobian(fwd, n)
    _unpack_state(fwd, n, x0)
    rhs = np.zeros(JF.shape[0])
    V, P, Q = _blocks(n)
    rhs[Q] = g.ravel()
    lam_dense = np.linalg.solve(JF.T, rhs)
    got = np.concatenate([lam["vx"][:, :, 1:-1].ravel(), lam["vy"][:, 1:-1, :].ravel(), lam["vz"][1:-1].ravel(),
                          lam["pt"].ravel(), lam["pf"].ravel()])
    assert np.abs(got - lam_dense).max() <= 1e-8 * np.abs(lam_dense).max()


def test_adjoint_gradient_matches_finite_differences():
    n = 8
    cfg, phi, logk0, sensors = _stage_setup(n, seed=3)
    fwd = adjoint.stage_forward(cfg.phys, n, n, n, phi, logk0, 1e-13)
    d_obs = fwd.f["pf"].ravel()[sensors] * 0.9 + 1e-3
    J0, g = adjoint.misfit(fwd.f["pf"], sensors, d_obs)
    lam, it, rho = adjoint.solve_adjoint(fwd, g, rtol=1e-13)
    grad = adjoint.gradient_log_k0(fwd, lam["pf"])
    rng = np.random.default_rng(7)
    cells = rng.choice(np.arange(n ** 3), size=4, replace=False)
    cells = np.concatenate([cells, sensors[:2]])
    h = 1e-4
    for c in cells:
        vals = []
        for sgn in (1.0, -1.0):
            m = logk0.copy().ravel()
            m[c] += sgn * h
            o = adjoint.stage_forward(cfg.phys, n, n, n, phi, m.reshape(logk0.shape), 1e-13)
            vals.append(adjoint.misfit(o.f["pf"], sensors, d_obs)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        gc = grad.ravel()[c]
        assert abs(gc - fd) <= 1e-6 * np.abs(grad).max() + 1e-4 * abs(fd), (c, gc, fd)
    assert np.abs(grad).max() > 0
