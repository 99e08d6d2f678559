"""Stage adjoint on the GPU: against the oracle's adjoint gradient, against
central finite differences of the misfit, and through torch.autograd."""
import numpy as np
import pytest

import oracle
from oracle import adjoint
from paper_2207_08716_amd import inputs

pytestmark = pytest.mark.gpu


def _problem(n, seed=5, ns=16):
    cfg = inputs.config_adjoint(n)
    phi = inputs.porosity_field(cfg)
    logk0 = np.log(inputs.k0_field(cfg))
    sensors = inputs.sensor_cells(seed, ns, cfg.shape)
    return cfg, phi, logk0, sensors


def _gpu_stage(cfg, phi, logk0, rtol):
    from paper_2207_08716_amd import grid
    g = grid.Grid(cfg.phys, cfg.nx, cfg.ny, cfg.nz, k0field=True)
    g.load_initial(phi, np.exp(logk0))
    g.set_log_k0(logk0)
    g.begin_step(False)
    g.refresh(1.0, 1.0)
    it, rho, ok = g.solve_linear(rtol, 2_000_000)
    assert ok
    return g


def test_adjoint_gradient_matches_oracle():
    n = 16
    cfg, phi, logk0, sensors = _problem(n)
    fwd = adjoint.stage_forward(cfg.phys, n, n, n, phi, logk0, 1e-13)
    d_obs = fwd.f["pf"].ravel()[sensors] * 0.8
    Jo, gbar = adjoint.misfit(fwd.f["pf"], sensors, d_obs)
    lam, _, _ = adjoint.solve_adjoint(fwd, gbar, rtol=1e-13)
    grad_o = adjoint.gradient_log_k0(fwd, lam["pf"])
    g = _gpu_stage(cfg, phi, logk0, 1e-13)
    J, grad, it, rho, ok = g.adjoint_stage(sensors, d_obs, rtol=1e-13)
    grad = grad.cpu().numpy()
    print("J", J, Jo, "iters", it, rho)
    assert ok
    assert abs(J - Jo) <= 1e-10 * abs(Jo)
    assert np.abs(grad - grad_o).max() <= 1e-8 * np.abs(grad_o).max()


def test_adjoint_gradient_matches_finite_differences():
    # forward and adjoint solves to 1e-11 (1e-13 is below the FP64 round-off
    # floor of the relative residual at this size); the finite-difference
    # noise is then ~1e-11 J / h, far below the 1e-6 tolerance
    n = 40
    rtol = 1e-11
    cfg, phi, logk0, sensors = _problem(n, seed=6, ns=64)
    g = _gpu_stage(cfg, phi, logk0, rtol)
    d_obs = g.get("pf").ravel()[sensors] * 0.8 + 1e-4
    J0, grad, it, rho, ok = g.adjoint_stage(sensors, d_obs, rtol=rtol)
    assert ok
    grad = grad.cpu().numpy().copy()
    rng = np.random.default_rng(7)
    cells = rng.choice(np.arange(n ** 3), size=8, replace=False)
    h = 1e-4
    gmax = np.abs(grad).max()
    for c in cells:
        vals = []
        for sgn in (1.0, -1.0):
            m = logk0.copy().ravel()
            m[c] += sgn * h
            g.reset_state(phi)
            g.set_log_k0(m.reshape(logk0.shape))
            g.begin_step(False)
            g.refresh(1.0, 1.0)
            _, _, ok = g.solve_linear(rtol, 2_000_000)
            assert ok
            vals.append(g.misfit(sensors, d_obs))
        fd = (vals[0] - vals[1]) / (2 * h)
        gc = grad.ravel()[c]
        print(c, gc, fd, flush=True)
        assert abs(gc - fd) <= 1e-6 * gmax + 1e-6 * abs(fd), (c, gc, fd)


def test_autograd_function():
    import torch
    from paper_2207_08716_amd import autograd as ag
    from paper_2207_08716_amd import grid
    n = 12
    cfg, phi, logk0, sensors = _problem(n, seed=8, ns=8)
    g = grid.Grid(cfg.phys, n, n, n, k0field=True)
    g.load_initial(phi, np.exp(logk0))
    prob = ag.StageProblem(g, phi, sensors, np.zeros(len(sensors)), rtol=1e-13)
    m = torch.tensor(logk0, dtype=torch.float64, device="cuda", requires_grad=True)
    J = ag.LogKMisfit.apply(m, prob)
    J.backward()
    grad = m.grad.detach().cpu().numpy()
    # directional derivative against central differences
    rng = np.random.default_rng(1)
    v = rng.standard_normal(logk0.shape)
    h = 1e-5
    with torch.no_grad():
        Jp = ag.LogKMisfit.apply(m + h * torch.tensor(v, device="cuda"), prob).item()
        Jm = ag.LogKMisfit.apply(m - h * torch.tensor(v, device="cuda"), prob).item()
    fd = (Jp - Jm) / (2 * h)
    dd = float((grad * v).sum())
    assert abs(dd - fd) <= 1e-6 * abs(fd), (dd, fd)


def test_autograd_backward_after_a_second_forward():
    """The gradient of a forward survives a later forward on the same problem
    (gradcheck, finite-difference probes and several losses do that)."""
    import torch
    from paper_2207_08716_amd import autograd as ag
    from paper_2207_08716_amd import grid
    n = 10
    cfg, phi, logk0, sensors = _problem(n, seed=9, ns=8)
    g = grid.Grid(cfg.phys, n, n, n, k0field=True)
    g.load_initial(phi, np.exp(logk0))
    prob = ag.StageProblem(g, phi, sensors, np.zeros(len(sensors)), rtol=1e-13)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(logk0.shape)
    m_a = torch.tensor(logk0, dtype=torch.float64, device="cuda", requires_grad=True)
    J_a = ag.LogKMisfit.apply(m_a, prob)
    m_b = torch.tensor(logk0 + 0.3 * v, dtype=torch.float64, device="cuda", requires_grad=True)
    J_b = ag.LogKMisfit.apply(m_b, prob)
    assert abs(J_a.item() - J_b.item()) > 1e-6 * abs(J_a.item())
    J_a.backward()
    grad = m_a.grad.detach().cpu().numpy()
    h = 1e-5
    with torch.no_grad():
        vt = torch.tensor(v, device="cuda")
        Jp = ag.LogKMisfit.apply(m_a + h * vt, prob).item()
        Jm = ag.LogKMisfit.apply(m_a - h * vt, prob).item()
    fd = (Jp - Jm) / (2 * h)
    dd = float((grad * v).sum())
    assert abs(dd - fd) <= 1e-6 * abs(fd), (dd, fd)
