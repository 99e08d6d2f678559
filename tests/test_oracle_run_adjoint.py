"""Pins of the oracle's adjoint of a Picard run (steps x stages): the stress
history's transposed operators against the oracle's forward code (dot-product
identities), and the gradient against central finite differences of the
whole run's misfit."""
import numpy as np

from oracle import Oracle, adjoint, field_shapes
from paper_2207_08716_amd import inputs


def _problem(n, seed=3):
    cfg = inputs.config_adjoint(n)
    phi = inputs.porosity_field(cfg)
    logk0 = np.log(inputs.k0_field(cfg))
    rng = np.random.default_rng(seed)
    sensors = np.sort(rng.choice(np.arange(n ** 3), size=6, replace=False))
    return cfg, phi, logk0, sensors, rng


def _stress_shapes(n):
    sh = field_shapes(n, n, n)
    return {"sxx": sh["cell"], "syy": sh["cell"], "szz": sh["cell"],
            "sxy": sh["sxy"], "sxz": sh["sxz"], "syz": sh["syz"]}


def _interior_v(rng, n):
    sh = field_shapes(n, n, n)
    v = {k: rng.standard_normal(sh[k]) for k in ("vx", "vy", "vz")}
    v["vx"][:, :, 0] = v["vx"][:, :, -1] = 0.0
    v["vy"][:, 0, :] = v["vy"][:, -1, :] = 0.0
    v["vz"][0] = v["vz"][-1] = 0.0
    return v


def _interior_s(rng, n):
    s = {k: rng.standard_normal(shp) for k, shp in _stress_shapes(n).items()}
    s["sxy"][:, 0, :] = s["sxy"][:, -1, :] = s["sxy"][:, :, 0] = s["sxy"][:, :, -1] = 0.0
    s["sxz"][0] = s["sxz"][-1] = s["sxz"][:, :, 0] = s["sxz"][:, :, -1] = 0.0
    s["syz"][0] = s["syz"][-1] = s["syz"][:, 0, :] = s["syz"][:, -1, :] = 0.0
    return s


def _dot(a, b):
    return sum(float(np.sum(a[k] * b[k])) for k in a)


def test_history_update_adjoint_is_transpose_of_forward():
    # So_new = a So + b E(V), computed by the oracle's own step set-up
    n = 5
    cfg, phi, logk0, _, rng = _problem(n)
    o = Oracle(cfg.phys, n, n, n, phi, np.exp(logk0))
    o.f["mus"][...] = 1e-3 * (1.0 + 0.5 * rng.random(o.f["mus"].shape))
    V, So, T = _interior_v(rng, n), _interior_s(rng, n), _interior_s(rng, n)
    for k in V:
        o.f[k][...] = V[k]
    for k in So:
        o.f[k][...] = So[k]
    o.step_index = 1
    o.begin_step()
    new = {k: o.f[k].copy() for k in So}
    vb, prev = adjoint.history_update_adjoint(o, T, o.f["mus"])
    lhs = _dot(T, new)
    rhs = _dot(vb, V) + _dot(prev, So)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + _dot(T, T) ** 0.5 * _dot(new, new) ** 0.5)


def test_history_divergence_adjoint_is_transpose_of_forward():
    # the momentum residual of a state with V = P = 0, no gravity and history
    # So is div(a So) on the interior faces
    n = 5
    cfg, phi, logk0, _, rng = _problem(n)
    ph = cfg.phys.replace(rhofg=0.0, rhosg=0.0)
    o = Oracle(ph, n, n, n, phi, np.exp(logk0))
    o.f["mus"][...] = 1e-3 * (1.0 + 0.5 * rng.random(o.f["mus"].shape))
    o.f["eta"][...] = 1.0
    So, W = _interior_s(rng, n), _interior_v(rng, n)
    for k in So:
        o.f[k][...] = So[k]
    fx, fy, fz, _, _ = o.residual()
    f = {"vx": fx, "vy": fy, "vz": fz}
    sb = adjoint.history_divergence_adjoint(o, W, o.f["mus"])
    lhs = _dot(W, f)
    rhs = _dot(sb, So)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + _dot(W, W) ** 0.5 * _dot(f, f) ** 0.5)


def test_transposed_solve_with_full_right_hand_side():
    # J_F lambda = rhs with all five blocks nonzero: the residual of the
    # forward stage at lambda (gravity off, no history) is J_F lambda + F(0)
    n = 4
    cfg, phi, logk0, _, rng = _problem(n)
    fwd = adjoint.stage_forward(cfg.phys, n, n, n, phi, logk0, 1e-12)
    rhs = {k: v for k, v in _interior_v(rng, n).items()}
    rhs["pt"] = rng.standard_normal((n, n, n))
    rhs["pf"] = rng.standard_normal((n, n, n))
    lam, it, rho = adjoint.solve_transposed(fwd, rhs, rtol=1e-12)
    # apply J_F: residual at lambda minus residual at 0, gravity off
    ph = cfg.phys.replace(rhofg=0.0, rhosg=0.0)
    a = Oracle(ph, n, n, n, phi, None)
    for k in ("lp", "kc", "eta", "mus", "mn"):
        a.f[k][...] = fwd.f[k]
    r0 = a.residual()
    for k in ("vx", "vy", "vz", "pt", "pf"):
        a.f[k][...] = lam[k]
    r1 = a.residual()
    names = ("vx", "vy", "vz", "pt", "pf")
    for q, k in enumerate(names):
        got = r1[q] - r0[q]
        scale = max(np.abs(rhs[kk]).max() for kk in names)
        assert np.abs(got - rhs[k]).max() <= 1e-9 * scale, k


def test_run_adjoint_matches_finite_differences():
    # two steps (the second with stress history) of two Picard stages; the
    # gradient reaches every term: porosity step, coefficients, old values,
    # history.  Forward solves to 1e-13, transposed solves to 1e-11.
    n, steps, stages = 6, 2, 2
    cfg, phi, logk0, sensors, rng = _problem(n)
    o, _ = adjoint.run_forward(cfg.phys, n, n, n, phi, logk0, steps, stages, 1e-13, record=False)
    d_obs = o.f["pf"].ravel()[sensors] * 0.9 + 1e-3
    J, grad = adjoint.run_adjoint(cfg.phys, n, n, n, phi, logk0, sensors, d_obs, steps, stages,
                                  1e-13, adj_rtol=1e-11)
    cells = list(rng.choice(np.arange(n ** 3), size=4, replace=False)) + list(sensors[:2])
    h = 1e-4
    gmax = np.abs(grad).max()
    assert gmax > 0
    for c in cells:
        vals = []
        for sgn in (1.0, -1.0):
            m = logk0.copy().ravel()
            m[c] += sgn * h
            vals.append(adjoint.run_misfit(cfg.phys, n, n, n, phi, m.reshape(logk0.shape), sensors, d_obs,
                                           steps, stages, 1e-13))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(grad.ravel()[c] - fd) <= 1e-7 * gmax + 1e-5 * abs(fd), (c, grad.ravel()[c], fd)


def test_run_adjoint_single_stage_equals_stage_adjoint():
    # one step of one stage: the run adjoint adds the porosity step and the
    # coefficient chain only through L, which the misfit does not see
    n = 6
    cfg, phi, logk0, sensors, rng = _problem(n)
    fwd = adjoint.stage_forward(cfg.phys, n, n, n, phi, logk0, 1e-13)
    d_obs = fwd.f["pf"].ravel()[sensors] * 0.9
    J1, g = adjoint.misfit(fwd.f["pf"], sensors, d_obs)
    lam, _, _ = adjoint.solve_adjoint(fwd, g, rtol=1e-12)
    grad1 = adjoint.gradient_log_k0(fwd, lam["pf"])
    J2, grad2 = adjoint.run_adjoint(cfg.phys, n, n, n, phi, logk0, sensors, d_obs, 1, 1, 1e-13, adj_rtol=1e-12)
    assert abs(J1 - J2) <= 1e-14 * abs(J1)
    assert np.abs(grad1 - grad2).max() <= 1e-9 * np.abs(grad1).max()
