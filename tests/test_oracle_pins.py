"""Pins of the FP64 oracle against results fixed by the paper or by mathematics.

Each test checks the oracle against something other than itself: a textbook
solver for a special case, a closed form, an exact invariant of the
discretisation, or a brute-force dense solve on a tiny grid.  A dropped term,
a wrong sign, a wrong index or a transposed operand anywhere in the residual
or the update should fail at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2207_08716_amd import inputs


def make(phys, n, phi=None, k0=None, lengths=(1.0, 1.0, 1.0)):
    phys = phys.replace(lx=lengths[0], ly=lengths[1], lz=lengths[2])
    if phi is None:
        phi = np.full((n, n, n), phys.phi0)
    return oracle.Oracle(phys, n, n, n, phi, k0)


# ---------------------------------------------------------------------------
# 1. PT converges to the implicit time step (article 1, eqs (12)-(16), Fig. 2)
# ---------------------------------------------------------------------------
def test_heat1d_pt_equals_backward_euler():
    """The Fig. 2 program's converged PT result is the backward-Euler step of
    the discrete heat equation with the end values held (tridiagonal solve)."""
    nx, lx = 200, 20.0
    dx = lx / (nx - 1)
    x = -lx / 2 + dx * np.arange(nx)
    dt = 1.0 / 50
    U = np.exp(-x ** 2)
    r = dt / dx ** 2
    for _ in range(4):
        Ut = U.copy()
        U_pt, it = oracle.heat1d_step(Ut, Ut, dx, dt, 1.0, 1e-14)
        ab = np.zeros((3, nx))
        ab[0, 2:] = -r
        ab[1, :] = 1 + 2 * r
        ab[2, :-2] = -r
        ab[1, 0] = ab[1, -1] = 1.0
        U_be = sla.solve_banded((1, 1), ab, Ut)
        assert it > 10
        assert np.max(np.abs(U_pt - U_be)) < 1e-12
        U = U_be


# ---------------------------------------------------------------------------
# 2. Fluid-pressure equation = a finite-volume diffusion step (eqs (18), (20))
# ---------------------------------------------------------------------------
def _fv_diffusion_matrix(K, h, c):
    """c I + L with L the cell-centred FV operator -div(Kf grad) on an n^3
    grid, face coefficient the mean of the two cells, no flux through the
    boundary.  Built independently of the oracle."""
    nz, ny, nx = K.shape
    idx = np.arange(K.size).reshape(K.shape)
    rows, cols, vals = [], [], []
    diag = np.full(K.size, c)
    for axis in range(3):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[axis] = slice(0, -1)
        sl_hi[axis] = slice(1, None)
        a = idx[tuple(sl_lo)].ravel()
        b = idx[tuple(sl_hi)].ravel()
        kf = 0.5 * (K[tuple(sl_lo)] + K[tuple(sl_hi)]).ravel() / h ** 2
        rows += [a, b]
        cols += [b, a]
        vals += [-kf, -kf]
        np.add.at(diag, a, kf)
        np.add.at(diag, b, kf)
    rows.append(np.arange(K.size))
    cols.append(np.arange(K.size))
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(K.size, K.size))


def test_fluid_pressure_step_is_fv_diffusion_solve():
    n = 8
    h = 1.0 / n
    rng = np.random.default_rng(11)
    phi = 0.01 * (1 + 0.5 * rng.random((n, n, n)))
    k0 = np.exp(0.5 * rng.standard_normal((n, n, n)))
    ph = inputs.Physics(mech_off=True, eta0=1e30, beta_phi=0.0, dt=5e-5, dtS=5e-5)
    o = make(ph, n, phi, k0)
    pf0 = rng.standard_normal((n, n, n))
    o.f["pf"][...] = pf0
    o.begin_step()
    o.refresh()
    # coefficient law k = k0 (phi/phi0)^3, eq (23)
    assert np.allclose(o.f["kc"], k0 * (phi / 0.01) ** 3, rtol=1e-13, atol=0)
    for _ in range(4000):
        nm = o.iteration(update_lp=False, norms=False)
    nm = o.iteration(update_lp=False, norms=True)
    assert nm["dPf"] < 1e-13
    c = ph.beta_d * ph.alpha / (ph.B * ph.dt)
    A = _fv_diffusion_matrix(o.f["kc"], h, c)
    # buoyancy flux q_z = -Kf (dPf/dz + (rho_f g - rho_bg g)) on interior z-faces
    buoy = ph.rhofg - (ph.rhofg * ph.phi0 + (1 - ph.phi0) * ph.rhosg)
    K = o.f["kc"]
    kfz = 0.5 * (K[:-1] + K[1:])
    src = np.zeros((n, n, n))
    src[:-1] += kfz * buoy / h     # -(q_top)/h contribution: q_top = -kf*buoy
    src[1:] -= kfz * buoy / h
    rhs = c * pf0.ravel() + src.ravel()
    ref = spla.spsolve(A.tocsc(), rhs).reshape(n, n, n)
    assert np.max(np.abs(o.f["pf"] - ref)) < 1e-9 * np.max(np.abs(ref))
    # velocities and total pressure frozen in this limit
    assert np.all(o.f["vz"] == 0) and np.all(o.f["pt"] == 0)


def _gauss1d_neumann(x, c, s2, s0):
    """1D Gaussian of variance-like width s2 on [0, 1] with zero-flux ends
    (method of images), normalised so that the free-space peak is
    (s0^2/s2)^(1/2)."""
    u = np.zeros_like(x)
    for m in (-2, -1, 0, 1, 2):
        u += np.exp(-(x - c - 2 * m) ** 2 / s2) + np.exp(-(x + c - 2 * m) ** 2 / s2)
    return u * np.sqrt(s0 ** 2 / s2)


def test_linear_limit_gaussian_diffusion_second_order():
    """Linear limit (V = 0, Pt fixed, 1/eta_phi = 0, beta_phi = 0, g = 0,
    uniform phi): dPf/dt = D lap Pf with D = k B / (alpha beta_d).  A Gaussian
    of width s0 spreads as exp(-r^2/(s0^2+4Dt)) (s0^2/(s0^2+4Dt))^(3/2), with
    images for the zero-flux walls.  With dt ~ h^2 the error falls by ~4 per
    halving of h (second order in space, first in time)."""
    errs = []
    s0 = 0.15
    for n in (12, 24):
        h = 1.0 / n
        ph = inputs.Physics(mech_off=True, eta0=1e30, beta_phi=0.0, rhofg=0.0, rhosg=0.0)
        D = ph.kmuf0 * ph.B / (ph.alpha * ph.beta_d)
        dt = 0.05 * h * h / D
        ph = ph.replace(dt=dt, dtS=dt)
        o = make(ph, n)
        xc = (np.arange(n) + 0.5) * h
        g0 = [_gauss1d_neumann(xc, 0.5, s0 ** 2, s0)] * 3
        o.f["pf"][...] = g0[2][:, None, None] * g0[1][None, :, None] * g0[0][None, None, :]
        nsteps = int(round(s0 ** 2 / (4 * D) / dt))
        for _ in range(nsteps):
            o.begin_step()
            o.refresh()
            for _ in range(120):
                o.iteration(update_lp=False)
            o.end_step()
        s2 = s0 ** 2 + 4 * D * nsteps * dt
        g = _gauss1d_neumann(xc, 0.5, s2, s0)
        exact = g[:, None, None] * g[None, :, None] * g[None, None, :]
        errs.append(np.sqrt(np.mean((o.f["pf"] - exact) ** 2)))
    ratio = errs[0] / errs[1]
    assert 3.2 < ratio < 5.0, (errs, ratio)


# ---------------------------------------------------------------------------
# 3. Buoyancy sign: a hydrostatic fluid has no Darcy flux (eqs (4), (20))
# ---------------------------------------------------------------------------
def test_hydrostatic_fluid_has_no_darcy_flux():
    n = 6
    ph = inputs.Physics()
    o = make(ph, n)
    o.refresh()
    rbg = ph.rhofg * ph.phi0 + (1 - ph.phi0) * ph.rhosg
    z = (np.arange(n) + 0.5) / n
    pf = (rbg - ph.rhofg) * z[:, None, None] * np.ones((n, n, n))
    o.f["pf"][...] = pf
    o.f["pfo"][...] = pf
    o.f["pt"][...] = pf
    o.f["pto"][...] = pf
    fx, fy, fz, rpt, rpf = o.residual()
    qx, qy, qz = o.last_fluxes()
    assert max(np.abs(qx).max(), np.abs(qy).max(), np.abs(qz).max()) < 1e-14
    assert np.abs(rpf).max() < 1e-13
    # and flipping the sign of the gradient gives a nonzero upward flux
    o.f["pf"][...] = -pf
    o.residual()
    qx, qy, qz = o.last_fluxes()
    assert qz[1:-1].min() > 0.1 * (rbg - ph.rhofg)


# ---------------------------------------------------------------------------
# 4. Maxwell visco-elastic stress (eqs (5), (21)) under steady simple shear
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("xi_target", [1.0, 0.05])
def test_maxwell_shear_stress_history(xi_target):
    n = 6
    ph = inputs.Physics()
    mus = ph.mu0 * ph.phi0 * ph.cmu
    dtS = mus / (ph.G * xi_target)
    ph = ph.replace(dtS=dtS)
    o = make(ph, n)
    o.refresh()
    gam = 0.7
    y = (np.arange(n) + 0.5) / n
    o.f["vx"][:, :, 1:-1] = gam * y[None, :, None]
    a = xi_target / (1 + xi_target)
    o.step_index = 1
    for m in range(1, 8):
        o.begin_step()
        sxy = o.f["sxy"]
        expect = mus * gam * (1 - a ** m)
        assert np.allclose(sxy[:, 1:-1, 1:-1], expect, rtol=1e-13, atol=0)
        # boundary edges carry no shear stress (free slip)
        assert np.all(sxy[:, 0, :] == 0) and np.all(sxy[:, :, 0] == 0)
        assert np.all(sxy[:, -1, :] == 0) and np.all(sxy[:, :, -1] == 0)


def test_maxwell_backward_euler_converges_to_exponential():
    """tau(t) = 2 mu edot (1 - exp(-G t / mu)) is the exact Maxwell response;
    the discrete stress history approaches it at first order in dtS."""
    n = 4
    ph = inputs.Physics()
    mus = ph.mu0 * ph.phi0 * ph.cmu
    gam = 1.0
    T = 2.0 * mus / ph.G
    errs = []
    for m in (8, 16, 32):
        dtS = T / m
        o = make(ph.replace(dtS=dtS), n)
        o.refresh()
        y = (np.arange(n) + 0.5) / n
        o.f["vx"][:, :, 1:-1] = gam * y[None, :, None]
        o.step_index = 1
        for _ in range(m):
            o.begin_step()
        exact = mus * gam * (1 - np.exp(-ph.G * T / mus))
        errs.append(abs(o.f["sxy"][1, 2, 2] - exact))
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3


# ---------------------------------------------------------------------------
# 5. Conservation: the flux divergences telescope (Sum div q = Sum div V = 0)
# ---------------------------------------------------------------------------
def test_divergences_telescope():
    n = 7
    rng = np.random.default_rng(3)
    phi = 0.01 * (1 + 0.5 * rng.random((n, n, n)))
    k0 = np.exp(rng.standard_normal((n, n, n)))
    ph = inputs.Physics(eta0=1e300)
    o = make(ph, n, phi, k0)
    o.refresh()
    o.f["vx"][:, :, 1:-1] = rng.standard_normal(o.f["vx"][:, :, 1:-1].shape)
    o.f["vy"][:, 1:-1, :] = rng.standard_normal(o.f["vy"][:, 1:-1, :].shape)
    o.f["vz"][1:-1] = rng.standard_normal(o.f["vz"][1:-1].shape)
    o.f["pf"][...] = rng.standard_normal((n, n, n))
    o.f["pfo"][...] = o.f["pf"]
    fx, fy, fz, rpt, rpf = o.residual()
    # Pt = Pto, Pf = Pfo, chi ~ 0: r_Pt = div V and r_Pf = div q
    assert abs(rpt.sum()) < 1e-13 * np.abs(rpt).sum()
    assert abs(rpf.sum()) < 1e-13 * np.abs(rpf).sum()


# ---------------------------------------------------------------------------
# 6. Structure of the discrete operator (probing the residual on 3^3)
# ---------------------------------------------------------------------------
def _unknown_slices(n):
    """Interior faces of Vx, Vy, Vz, then all Pt, all Pf cells."""
    return [("vx", (slice(None), slice(None), slice(1, -1))),
            ("vy", (slice(None), slice(1, -1), slice(None))),
            ("vz", (slice(1, -1), slice(None), slice(None))),
            ("pt", (slice(None),) * 3), ("pf", (slice(None),) * 3)]


def _pack_state(o, n):
    return np.concatenate([o.f[name][sl].ravel() for name, sl in _unknown_slices(n)])


def _unpack_state(o, n, x):
    off = 0
    for name, sl in _unknown_slices(n):
        view = o.f[name][sl]
        m = view.size
        o.f[name][sl] = x[off:off + m].reshape(view.shape)
        off += m


def _residual_vector(o, n):
    fx, fy, fz, rpt, rpf = o.residual()
    return np.concatenate([fx[:, :, 1:-1].ravel(), fy[:, 1:-1, :].ravel(), fz[1:-1].ravel(),
                           rpt.ravel(), rpf.ravel()])


def _jacobian(o, n):
    x0 = _pack_state(o, n)
    F0 = _residual_vector(o, n)
    J = np.zeros((F0.size, x0.size))
    for m in range(x0.size):
        e = x0.copy()
        e[m] += 1.0
        _unpack_state(o, n, e)
        J[:, m] = _residual_vector(o, n) - F0
    _unpack_state(o, n, x0)
    return J, F0


def _blocks(n):
    nv = 3 * (n - 1) * n * n
    nc = n ** 3
    return slice(0, nv), slice(nv, nv + nc), slice(nv + nc, nv + 2 * nc)


def _tiny_problem(n=3, seed=5, **kw):
    rng = np.random.default_rng(seed)
    phi = 0.01 * (1 + 0.8 * rng.random((n, n, n)))
    k0 = np.exp(0.5 * rng.standard_normal((n, n, n)))
    ph = inputs.Physics(**kw)
    o = make(ph, n, phi, k0, lengths=(1.0, 1.3, 0.8))
    o.f["pt"][...] = 0.1 * rng.standard_normal((n, n, n))
    o.f["pf"][...] = 0.1 * rng.standard_normal((n, n, n))
    o.begin_step()
    o.f["pf"][...] += 0.05          # Pf > Pt in part of the cells: weakening
    o.refresh()
    o.f["mus"][...] *= 1.0 + rng.random((n, n, n))   # heterogeneous shear viscosity
    o.f["pt"][...] = 0
    o.f["pf"][...] = 0
    return o


def test_operator_block_structure():
    n = 3
    o = _tiny_problem(n)
    J, F0 = _jacobian(o, n)
    V, P, Q = _blocks(n)
    JVV = J[V, V]
    # viscous operator: symmetric and negative semi-definite (Dt M D form)
    assert np.allclose(JVV, JVV.T, rtol=0, atol=1e-12 * np.abs(JVV).max())
    ev = np.linalg.eigvalsh(0.5 * (JVV + JVV.T))
    assert ev.max() < 1e-10 * np.abs(ev).max()
    # momentum carries -grad Pt and r_Pt carries +div V, and the discrete
    # gradient is minus the transpose of the discrete divergence, so the two
    # coupling blocks are transposes of each other
    assert np.allclose(J[V, P], J[P, V].T, rtol=0, atol=1e-12 * np.abs(J[P, V]).max())
    assert np.abs(J[V, P]).max() > 0
    # momentum does not see Pf; total-pressure residual sees V only via div V
    assert np.all(J[V, Q] == 0)
    assert np.all(J[Q, V] == 0)
    # pressure-pressure couplings are symmetric (equal off-diagonal terms)
    assert np.allclose(J[P, Q], J[Q, P].T, rtol=1e-13, atol=0)
    assert np.count_nonzero(J[P, P] - np.diag(np.diag(J[P, P]))) == 0
    JQQ = J[Q, Q]
    assert np.allclose(JQQ, JQQ.T, rtol=1e-13, atol=1e-13 * np.abs(JQQ).max())


def test_pt_fixed_point_is_direct_solve():
    """Brute force: the converged linear PT iteration equals the dense LU
    solution of the probed linear system (frozen coefficients)."""
    n = 4
    o = _tiny_problem(n, seed=9, dt=1e-4, dtS=1e-4)
    J, F0 = _jacobian(o, n)
    x_direct = np.linalg.solve(J, -F0)
    for _ in range(8000):
        o.iteration(update_lp=False)
    x_pt = _pack_state(o, n)
    scale = np.abs(x_direct).max()
    assert np.max(np.abs(x_pt - x_direct)) < 1e-9 * scale


# ---------------------------------------------------------------------------
# 7. Mirror symmetry of a symmetric set-up
# ---------------------------------------------------------------------------
def test_mirror_symmetry():
    cfg = inputs.config_parity(10)
    cfg.noise_seed = None
    f = inputs.initial_fields(cfg)
    o = oracle.Oracle(cfg.phys, cfg.nx, cfg.ny, cfg.nz, f["phi"], None)
    o.begin_step()
    o.iterate(150)
    for name in ("pt", "pf", "lp"):
        a = o.f[name]
        s = np.abs(a).max()
        assert np.abs(a - a[:, :, ::-1]).max() <= 1e-12 * s
        assert np.abs(a - a[:, ::-1, :]).max() <= 1e-12 * s
    vx, vy, vz = o.f["vx"], o.f["vy"], o.f["vz"]
    assert np.abs(vx + vx[:, :, ::-1]).max() <= 1e-12 * np.abs(vz).max()
    assert np.abs(vy + vy[:, ::-1, :]).max() <= 1e-12 * np.abs(vz).max()
    assert np.abs(vz - vz[:, :, ::-1]).max() <= 1e-12 * np.abs(vz).max()
    assert np.abs(vz).max() > 0


# ---------------------------------------------------------------------------
# 8. Coefficient refresh special cases (eqs (23)-(26))
# ---------------------------------------------------------------------------
def test_decompaction_weakening_switch():
    n = 4
    ph = inputs.Physics()
    rng = np.random.default_rng(2)
    phi = 0.01 * (1 + rng.random((n, n, n)))
    o = make(ph, n, phi)
    o.f["pf"][...] = 1.0
    o.f["pt"][...] = 0.0
    o.refresh()
    weak = o.f["eta"].copy()
    o2 = make(ph, n, phi)
    o2.refresh()
    assert np.allclose(weak * ph.R0, o2.f["eta"], rtol=1e-15, atol=0)
    # eta_phi = eta0 mu (phi0/phi): unit at phi0 without weakening
    o3 = make(ph, n)
    o3.refresh()
    assert np.allclose(o3.f["eta"], 1.0, rtol=1e-15, atol=0)
    # Pf == Pt (tie) does not weaken
    o4 = make(ph, n, phi)
    o4.f["pf"][...] = 0.3
    o4.f["pt"][...] = 0.3
    o4.refresh()
    assert np.array_equal(o4.f["eta"], o2.f["eta"])


def test_drucker_prager_cap():
    cfg = inputs.config_parity(8)
    f = inputs.initial_fields(cfg)
    base = oracle.Oracle(cfg.phys, 8, 8, 8, f["phi"], None)
    huge = oracle.Oracle(cfg.phys.replace(dpcap=True, coh=1e30), 8, 8, 8, f["phi"], None)
    for o in (base, huge):
        o.begin_step()
        o.iterate(60)
    for name in ("vx", "vz", "pt", "pf", "lp", "mus"):
        assert np.array_equal(base.f[name], huge.f[name])
    # a small cohesion makes cells yield: Mn_new <= Mn tau_y / tau_II there
    weak = oracle.Oracle(cfg.phys.replace(dpcap=True, coh=1e-6, tau_y_min=1e-9), 8, 8, 8, f["phi"], None)
    weak.begin_step()
    weak.iterate(45)
    tii = weak.tau_ii()
    pt, pf = weak.f["pt"].copy(), weak.f["pf"].copy()
    mn_old = weak.f["mn"].copy()
    weak.refresh(r_eta=1.0, r_mu=1.0)
    ty = np.maximum(1e-6 * np.cos(np.pi / 6) + (pt - pf) * np.sin(np.pi / 6), 1e-9)
    yielded = tii > ty
    assert yielded.mean() > 0.05
    assert np.all(weak.f["mn"][yielded] <= mn_old[yielded] * ty[yielded] / tii[yielded] * (1 + 1e-14))
    # elsewhere the viscous value, unless an earlier cut left Mn on the yield
    # surface: min(mu0, Mn tau_y / tau_II)
    expect = np.minimum(cfg.phys.mu0, mn_old * ty / tii)
    assert np.allclose(weak.f["mn"][~yielded], expect[~yielded], rtol=1e-14, atol=0)


def test_power_law_viscosity_limits():
    """eq (24): mu_s -> mu0 for tau_II << tau0; halves at tau_II = tau0 (n = 3)."""
    cfg = inputs.config_parity(8)
    f = inputs.initial_fields(cfg)
    o = oracle.Oracle(cfg.phys.replace(powerlaw=True), 8, 8, 8, f["phi"], None)
    o.begin_step()
    o.iterate(30)
    tii = o.tau_ii()
    mn_old = o.f["mn"].copy()
    o.refresh(r_eta=1.0, r_mu=1.0)
    expect = 1.0 / (1.0 + (tii / 0.04) ** 2)
    assert np.allclose(o.f["mn"], expect, rtol=1e-13, atol=0)
    del mn_old


def test_log_space_relaxation_of_the_refresh():
    """After the first refresh of a run, eta_phi and Mn relax in log space:
    x = x_new^r x_old^(1-r).  At phi = phi0, Pf <= Pt and no stress
    dependence, eta_new = eta0 Mn_old and Mn_new = mu0, so from chosen old
    values the relaxed ones follow in closed form (r = 0.5, 0.1 and 1)."""
    n = 4
    ph = inputs.Physics()
    for r_eta, r_mu in ((0.5, 0.1), (1.0, 1.0), (0.25, 0.75)):
        o = make(ph, n)                       # phi = phi0 everywhere
        o.refresh()                           # the first refresh takes new values
        eta_old, mn_old = 4.0, 0.25
        o.f["eta"][...] = eta_old
        o.f["mn"][...] = mn_old
        o.refresh(r_eta=r_eta, r_mu=r_mu)
        eta_new = ph.eta0 * mn_old
        assert np.allclose(o.f["eta"], eta_new ** r_eta * eta_old ** (1 - r_eta), rtol=1e-14, atol=0)
        assert np.allclose(o.f["mn"], ph.mu0 ** r_mu * mn_old ** (1 - r_mu), rtol=1e-14, atol=0)


def test_stress_invariant_closed_forms():
    """tau_II of eq (21)'s stresses (without the numerical compressibility
    term), as the refresh uses it, for fields whose invariant is known in
    closed form, with uniform mu_s (b = 2 mu/(1+xi), a = xi/(1+xi)):
    pure shear V = (e x, -e y, 0): tau_xx = b e = -tau_yy, tau_II = b e;
    simple shear V = (g y, 0, 0): tau_xy = b g/2 on interior edges, so
    tau_II = b g/2 in cells whose four xy-edges are interior;
    history only (V = 0): So_xx = s = -So_yy gives tau_II = a s, and a uniform
    So_xy = t on interior edges gives a t in the inner cells."""
    cfg = inputs.config_parity(8)
    ph = cfg.phys
    n = 8
    f = inputs.initial_fields(cfg)
    dx, dy = ph.lx / n, ph.ly / n
    mu = ph.mu0 * ph.phi0 * ph.cmu
    xi = mu / (ph.G * ph.dtS)
    b, a = 2.0 * mu / (1.0 + xi), xi / (1.0 + xi)
    inner = (slice(None), slice(1, n - 1), slice(1, n - 1))

    o = oracle.Oracle(ph, n, n, n, f["phi"], None)
    e = 0.3
    o.f["vx"][...] = e * (np.arange(n + 1) * dx)[None, None, :]
    o.f["vy"][...] = -e * (np.arange(n + 1) * dy)[None, :, None]
    assert np.allclose(o.tau_ii(), b * e, rtol=1e-13, atol=0)

    o = oracle.Oracle(ph, n, n, n, f["phi"], None)
    g = 0.7
    o.f["vx"][...] = g * ((np.arange(n) + 0.5) * dy)[None, :, None]
    assert np.allclose(o.tau_ii()[inner], 0.5 * b * g, rtol=1e-13, atol=0)

    o = oracle.Oracle(ph, n, n, n, f["phi"], None)
    s_, t_ = 0.2, 0.05
    o.f["sxx"][...] = s_
    o.f["syy"][...] = -s_
    assert np.allclose(o.tau_ii(), a * s_, rtol=1e-13, atol=0)
    o.f["sxx"][...] = 0.0
    o.f["syy"][...] = 0.0
    o.f["sxy"][...] = t_
    assert np.allclose(o.tau_ii()[inner], a * t_, rtol=1e-13, atol=0)


# ---------------------------------------------------------------------------
# 9. Seeded inputs are reproducible and have the stated statistics
# ---------------------------------------------------------------------------
def test_inputs_reproducible():
    a = inputs.initial_fields(inputs.config_fp64_picard(16))
    b = inputs.initial_fields(inputs.config_fp64_picard(16))
    assert np.array_equal(a["phi"], b["phi"]) and np.array_equal(a["k0"], b["k0"])
    c = inputs.config_parity(32)
    phi = inputs.porosity_field(c)
    assert 2.5 < phi.max() / c.phys.phi0 < 3.0 * (1 + 1e-3)
    g = inputs.gaussian_random_field((32, 32, 32), (1, 1, 1), 0.1, 4)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12


def test_porosity_step_closed_forms():
    """Eq (22) in log space, L = ln(1 - phi): d L/dt = -(1/(1-phi)) d^s phi/dt
    = beta_phi d(Pt - Pf)/dt + (Pt - Pf)/eta_phi - V.grad(1-phi) terms.
    (i) with a constant effective pressure Pt - Pf = D, no storage change and
    V = 0, L grows linearly, L(t) = L0 + t D/eta (the exact solution; the
    explicit step is exact); (ii) a uniform pressure change dPf with Pt fixed
    lowers L by beta_phi dPf; (iii) a uniform velocity U in x over a solid
    fraction linear in x gives the advection rate U ds/dx away from the
    boundaries."""
    n = 6
    ph = inputs.Physics()
    o = make(ph, n)
    eta = 2.5
    o.f["eta"][...] = eta
    D = 0.3
    o.f["pt"][...] = 1.0 + D
    o.f["pf"][...] = 1.0
    o.f["pto"][...] = o.f["pt"]
    o.f["pfo"][...] = o.f["pf"]
    L0 = o.f["lp"].copy()
    for step in range(1, 4):
        o.f["lpo"][...] = o.f["lp"]
        o.porosity_step()
        assert np.allclose(o.f["lp"], L0 + step * ph.dt * D / eta, rtol=0, atol=1e-15)
    # (ii) storage: Pf - Pfo = dp, Pt = Pto, Pt = Pf (no viscous term)
    o.f["lp"][...] = L0
    o.f["lpo"][...] = L0
    dp = 0.05
    o.f["pt"][...] = 1.0
    o.f["pto"][...] = 1.0
    o.f["pfo"][...] = 1.0 - dp
    o.f["pf"][...] = 1.0
    o.f["pt"][...] = 1.0
    o.porosity_step()
    assert np.allclose(o.f["lp"], L0 - ph.beta_phi * dp, rtol=0, atol=1e-15)
    # (iii) advection: s = 1 - phi linear in x, Vx = U on interior x-faces
    x = (np.arange(n) + 0.5) / n
    s = 0.98 + 0.01 * x
    o.f["lp"][...] = np.log(s)[None, None, :]
    o.f["lpo"][...] = o.f["lp"]
    o.f["pto"][...] = o.f["pt"]
    o.f["pfo"][...] = o.f["pf"]
    U = 0.7
    o.f["vx"][...] = U
    o.f["vx"][:, :, 0] = 0.0
    o.f["vx"][:, :, -1] = 0.0
    Lb = o.f["lp"].copy()
    o.porosity_step()
    rate = -(o.f["lp"] - Lb) / ph.dt
    assert np.allclose(rate[:, :, 1:-1], U * 0.01, rtol=1e-12, atol=0)
