"""Adjoint of one linear Picard stage, FP64 CPU reference.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Problem.  Within a Picard stage the coefficients (k/mu_f = K, eta_phi, mu_s)
and the porosity are frozen and the stage solves the linear system
F(x; K) = 0 for x = (V, Pt, Pf), F = (momentum residual f, r_Pt, r_Pf) of
eqs (17)-(20).  The misfit J = 1/2 sum_s (Pf(x)_s - d_s)^2 over sensor cells s
depends on m = ln k0 through K = k0 (phi/phi0)^3.  With lambda solving
J_F^T lambda = dJ/dx, dJ/dm_c = -lambda^T dF/dm_c, and dF/dm_c = K_c dF/dK_c
touches only the Darcy flux in r_Pf.

The residual Jacobian J_F of this discretisation is symmetric (momentum rows
carry -grad Pt, the total-pressure row carries +div V, the Pt-Pf couplings are
equal, the viscous and Darcy operators are symmetric), so J_F^T = J_F and the
adjoint is the forward stage operator with a different right-hand side.  Here
that system is solved by the oracle's own, unchanged PT stage solve: with
gravity off and no stress history the stage residual at x = 0 reduces to the
old-value terms, so choosing
    Pto = alpha Pfo,   Pfo = g dt / (beta_d alpha (1/B - alpha))
makes F(0) = (0, 0, -g) with g = dJ/dPf, and the converged state is lambda.
"""
from __future__ import annotations

import numpy as np

from . import Oracle, field_shapes


def misfit(pf: np.ndarray, sensors: np.ndarray, d_obs: np.ndarray):
    """J and dJ/dPf (a cell field) for sensor cells given as linear indices."""
    v = pf.ravel()[sensors]
    r = v - d_obs
    g = np.zeros(pf.size)
    g[sensors] = r
    return 0.5 * float(np.dot(r, r)), g.reshape(pf.shape)


def solve_transposed(fwd: Oracle, rhs: dict, rtol: float = 1e-12, max_iter: int = 400000,
                     coef: dict = None):
    """lambda = (vx, vy, vz, pt, pf) with J_F lambda = rhs, rhs a dict of the
    same five fields (momentum rows on the faces, r_Pt and r_Pf rows in the
    cells), for the stage whose frozen coefficients and porosity are those
    of `fwd` (or of `coef`: lp, kc, eta, mus, mn arrays).

    J_F is symmetric, so this is the stage's own linear system with another
    right-hand side, solved by the oracle's unchanged PT stage solve: gravity
    off and no stress history make F affine with F(0) = (fs, r_Pt(0),
    r_Pf(0)); the momentum source fs = -rhs_V and old pressures solving
        beta_d/dt (-Pto + alpha Pfo)        = -rhs_Pt
        beta_d/dt (alpha Pto - (alpha/B) Pfo) = -rhs_Pf
    give F(0) = -rhs, so the converged state solves J_F lambda = rhs."""
    ph0 = fwd.phys
    ph = ph0.replace(rhofg=0.0, rhosg=0.0)
    src = coef if coef is not None else fwd.f
    a = Oracle(ph, fwd.nx, fwd.ny, fwd.nz, 1.0 - np.exp(src["lp"]), None)
    for name in ("lp", "kc", "eta", "mus", "mn"):
        a.f[name][...] = src[name]
    bd, al, ab = ph0.beta_d, ph0.alpha, ph0.alpha / ph0.B
    pfo = (rhs["pf"] + al * rhs["pt"]) * ph0.dt / (bd * (ab - al * al))
    a.f["pfo"][...] = pfo
    a.f["pto"][...] = al * pfo + rhs["pt"] * ph0.dt / bd
    a.set_momentum_source(-rhs["vx"], -rhs["vy"], -rhs["vz"])
    a.refreshed = True          # coefficients are given, never refreshed here
    a.ref = None
    it, rho = a.solve_linear(rtol, max_iter)
    return {k: a.f[k].copy() for k in ("vx", "vy", "vz", "pt", "pf")}, it, rho


def _zero_rhs(o: Oracle) -> dict:
    sh = field_shapes(o.nx, o.ny, o.nz)
    return {"vx": np.zeros(sh["vx"]), "vy": np.zeros(sh["vy"]), "vz": np.zeros(sh["vz"]),
            "pt": np.zeros(sh["cell"]), "pf": np.zeros(sh["cell"])}


def solve_adjoint(fwd: Oracle, g_pf: np.ndarray, rtol: float = 1e-12, max_iter: int = 400000):
    """lambda = (lam_vx, lam_vy, lam_vz, lam_pt, lam_pf) with J_F lambda = (0, 0, g)
    for the stage whose frozen coefficients and porosity are those of `fwd`."""
    rhs = _zero_rhs(fwd)
    rhs["pf"] = np.asarray(g_pf, dtype=np.float64)
    return solve_transposed(fwd, rhs, rtol, max_iter)


def gradient_log_k0(fwd: Oracle, lam_pf: np.ndarray) -> np.ndarray:
    """dJ/d(ln k0) per cell from the adjoint fluid pressure.

    The Darcy flux through the face between a lower cell L and an upper cell H
    is q = -(K_L + K_H)/2 * ((Pf_H - Pf_L)/h + b) (b the buoyancy term on
    z-faces, 0 otherwise), and r_Pf carries +q/h in L and -q/h in H.  Hence
    d(lambda^T F)/dK_c = sum over c's interior faces of
    -(1/2) ((Pf_H - Pf_L)/h + b) (lam_L - lam_H)/h, and
    dJ/dm_c = -K_c d(lambda^T F)/dK_c."""
    ph = fwd.phys
    K = fwd.f["kc"]
    pf = fwd.f["pf"]
    nz, ny, nx = K.shape
    h = (ph.lz / nz, ph.ly / ny, ph.lx / nx)
    buoy = ph.rhofg - (ph.rhofg * ph.phi0 + (1.0 - ph.phi0) * ph.rhosg)
    dphi = np.zeros_like(K)   # d(lambda^T F)/dK
    for axis in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        grad = (pf[hi] - pf[lo]) / h[axis] + (buoy if axis == 0 else 0.0)
        dl = (lam_pf[lo] - lam_pf[hi]) / h[axis]
        term = -0.5 * grad * dl
        dphi[lo] += term
        dphi[hi] += term
    return -K * dphi


def stage_forward(phys, nx, ny, nz, phi, logk0, rtol, max_iter=400000):
    """One linear Picard stage from the initial state: refresh (k from
    exp(logk0)), then the linear solve.  Returns the oracle."""
    o = Oracle(phys, nx, ny, nz, phi, np.exp(logk0))
    o.begin_step()
    o.refresh(1.0, 1.0)
    o.solve_linear(rtol, max_iter)
    return o


# ---------------------------------------------------------------------------
# Adjoint of a run of Picard steps (steps x stages), through the refresh, the
# porosity step, the old values and the stress history.
#
# Forward, per physical step n (history update from the run's second step on):
#   So_n = a So_{n-1} + b E(V_{n-1})          (begin_step; E = deviatoric strain
#                                               rate, edges 1/2(dVx/dy + dVy/dx))
#   Pto, Pfo, Lo = Pt, Pf, L at the end of step n-1
#   per stage p:  c = (K = k0 (phi/phi0)^3, eta = eta0 Mn (phi0/phi) R, s = 1-phi)
#                 from L_{p-1} (refresh without relaxation);
#                 x_p solves F(x; c, Pto, Pfo, So_n) = 0 (linear stage);
#                 L_p = Lo - dt Phi(x_p, eta, s, Pto, Pfo)       (eq (22)).
# J = 1/2 sum_s (Pf_s - d_s)^2 at the end of the run, m = ln k0.
# Reverse: for each stage, the porosity step's adjoint gives the right-hand
# side of the transposed stage solve J_F^T lambda = xbar (J_F symmetric);
# then theta_bar = -lambda^T dF/dtheta for K, chi = 1/(eta s), s (buoyancy),
# Pto, Pfo and the history term div(a So); the coefficient chain maps
# K_bar, eta_bar, s_bar to L_bar of the stage's incoming porosity and to m.
# The switch R (Pf > Pt at refresh) is piecewise constant: no derivative.
# Needs the Newtonian law (no power law, no cap: mu_s then never changes).
# ---------------------------------------------------------------------------

def _sl(axis, a, b):
    s = [slice(None)] * 3
    s[axis] = slice(a, b)
    return tuple(s)


def _spacings(o: Oracle):
    ph = o.phys
    return {2: ph.lx / o.nx, 1: ph.ly / o.ny, 0: ph.lz / o.nz}


_FACE = {2: "vx", 1: "vy", 0: "vz"}


def porosity_step_adjoint(o: Oracle, rec: dict, Lbar: np.ndarray, xbar: dict, acc: dict):
    """Adjoint of L_p = Lo - dt Phi.  Adds to xbar (pt, pf, V faces) and to
    acc['pto'], acc['pfo'], acc['lo']; returns (eta_bar, s_bar) of Phi."""
    ph = o.phys
    h = _spacings(o)
    s = np.exp(rec["lp"])
    eta = rec["eta"]
    phib = -ph.dt * Lbar
    c1 = ph.beta_phi / ph.dt + 1.0 / eta
    xbar["pf"] += phib * c1
    xbar["pt"] -= phib * c1
    acc["pfo"] -= phib * ph.beta_phi / ph.dt
    acc["pto"] += phib * ph.beta_phi / ph.dt
    acc["lo"] += Lbar
    eta_bar = -phib * (rec["pf"] - rec["pt"]) / eta ** 2
    s_bar = np.zeros_like(s)
    # advection: an interior face between cells lo and hi adds
    # 1/2 V (s_hi - s_lo)/h to the rate of both cells
    for axis in (2, 1, 0):
        lo, hi = _sl(axis, 0, -1), _sl(axis, 1, None)
        w = 0.5 * (phib[lo] + phib[hi]) / h[axis]
        V = rec[_FACE[axis]][_sl(axis, 1, -1)]
        xbar[_FACE[axis]][_sl(axis, 1, -1)] += w * (s[hi] - s[lo])
        s_bar[hi] += w * V
        s_bar[lo] -= w * V
    return eta_bar, s_bar


def stage_parameter_adjoint(o: Oracle, rec: dict, lam: dict, acc: dict):
    """theta_bar = -lambda^T dF/dtheta for the stage's K, chi, s (buoyancy),
    Pto, Pfo and history term; returns (K_bar, chi_bar, s_bar) and adds the
    history term's adjoint (-lambda_V) to acc['fo']."""
    ph = o.phys
    h = _spacings(o)
    pf, pt = rec["pf"], rec["pt"]
    buoy = ph.rhofg - (ph.rhofg * ph.phi0 + (1.0 - ph.phi0) * ph.rhosg)
    # Darcy: an interior face carries q = -(K_lo + K_hi)/2 ((Pf_hi - Pf_lo)/h + b)
    # and r_Pf has +q/h in lo, -q/h in hi
    dFdK = np.zeros_like(pf)
    for axis in (2, 1, 0):
        lo, hi = _sl(axis, 0, -1), _sl(axis, 1, None)
        grad = (pf[hi] - pf[lo]) / h[axis] + (buoy if axis == 0 else 0.0)
        term = -0.5 * grad * (lam["pf"][lo] - lam["pf"][hi]) / h[axis]
        dFdK[lo] += term
        dFdK[hi] += term
    K_bar = -dFdK
    # chi couples (Pt - Pf) into r_Pt and (Pf - Pt) into r_Pf
    chi_bar = -(lam["pt"] - lam["pf"]) * (pt - pf)
    # buoyancy on interior z-faces: -(1/2 (rho g_lo + rho g_hi) - rho_bg g),
    # rho g = rhof g (1 - s) + rhos g s
    s_bar = np.zeros_like(pf)
    lz = lam["vz"][1:-1]
    s_bar[:-1] += 0.5 * (ph.rhosg - ph.rhofg) * lz
    s_bar[1:] += 0.5 * (ph.rhosg - ph.rhofg) * lz
    bd, al, ab = ph.beta_d, ph.alpha, ph.alpha / ph.B
    acc["pto"] += bd / ph.dt * (lam["pt"] - al * lam["pf"])
    acc["pfo"] += bd / ph.dt * (ab * lam["pf"] - al * lam["pt"])
    for k in ("vx", "vy", "vz"):
        acc["fo"][k] -= lam[k]
    return K_bar, chi_bar, s_bar


def coefficient_adjoint(o: Oracle, rec: dict, K_bar, eta_bar, s_bar, chi_bar):
    """Chain of the refresh: K = k0 (phi/phi0)^3, eta = eta0 Mn (phi0/phi) R,
    chi = 1/(eta s), s = exp(L), phi = 1 - s.  Returns (L_bar, m_bar)."""
    s = np.exp(rec["lp"])
    phi = 1.0 - s
    K, eta = rec["kc"], rec["eta"]
    eta_t = eta_bar - chi_bar / (eta * eta * s)
    s_t = s_bar - chi_bar / (eta * s * s)
    L_bar = -3.0 * K_bar * K * s / phi + eta_t * eta * s / phi + s_t * s
    return L_bar, K_bar * K


def _edge_coefs(o: Oracle, mus: np.ndarray):
    """Maxwell a, b at cells and at the interior edges (xy, xz, yz), as the
    stresses take them (edge viscosity = mean of the four cells)."""
    ph = o.phys
    gdt = ph.G * ph.dtS

    def ab(mu):
        xi = mu / gdt
        return xi / (1.0 + xi), 2.0 * mu / (1.0 + xi)
    m = mus
    exy = 0.25 * (m[:, :-1, :-1] + m[:, :-1, 1:] + m[:, 1:, :-1] + m[:, 1:, 1:])
    exz = 0.25 * (m[:-1, :, :-1] + m[:-1, :, 1:] + m[1:, :, :-1] + m[1:, :, 1:])
    eyz = 0.25 * (m[:-1, :-1, :] + m[:-1, 1:, :] + m[1:, :-1, :] + m[1:, 1:, :])
    return {"c": ab(m), "xy": ab(exy), "xz": ab(exz), "yz": ab(eyz)}


def history_divergence_adjoint(o: Oracle, fo_bar: dict, mus: np.ndarray) -> dict:
    """Adjoint of the history term div(a So) in the momentum rows: given the
    adjoint w of that face term, returns a * D^T w for the six stress-history
    components (boundary edges, which carry no stress, get zero)."""
    h = _spacings(o)
    dx, dy, dz = h[2], h[1], h[0]
    wx, wy, wz = (np.array(fo_bar[k]) for k in ("vx", "vy", "vz"))
    wx[:, :, 0] = wx[:, :, -1] = 0.0
    wy[:, 0, :] = wy[:, -1, :] = 0.0
    wz[0] = wz[-1] = 0.0
    co = _edge_coefs(o, mus)
    ac = co["c"][0]
    out = {}
    out["sxx"] = ac * (wx[:, :, :-1] - wx[:, :, 1:]) / dx
    out["syy"] = ac * (wy[:, :-1, :] - wy[:, 1:, :]) / dy
    out["szz"] = ac * (wz[:-1] - wz[1:]) / dz
    nz, ny, nx = mus.shape
    sxy = np.zeros((nz, ny + 1, nx + 1))
    sxy[:, 1:-1, 1:-1] = co["xy"][0] * ((wx[:, :-1, 1:-1] - wx[:, 1:, 1:-1]) / dy
                                        + (wy[:, 1:-1, :-1] - wy[:, 1:-1, 1:]) / dx)
    sxz = np.zeros((nz + 1, ny, nx + 1))
    sxz[1:-1, :, 1:-1] = co["xz"][0] * ((wx[:-1, :, 1:-1] - wx[1:, :, 1:-1]) / dz
                                        + (wz[1:-1, :, :-1] - wz[1:-1, :, 1:]) / dx)
    syz = np.zeros((nz + 1, ny + 1, nx))
    syz[1:-1, 1:-1, :] = co["yz"][0] * ((wy[:-1, 1:-1, :] - wy[1:, 1:-1, :]) / dz
                                        + (wz[1:-1, :-1, :] - wz[1:-1, 1:, :]) / dy)
    out["sxy"], out["sxz"], out["syz"] = sxy, sxz, syz
    return out


def history_update_adjoint(o: Oracle, so_bar: dict, mus: np.ndarray):
    """Adjoint of So_n = a So_{n-1} + b E(V): returns (V_bar faces dict,
    So_bar of the previous history)."""
    h = _spacings(o)
    dx, dy, dz = h[2], h[1], h[0]
    co = _edge_coefs(o, mus)
    bc = co["c"][1]
    nz, ny, nx = mus.shape
    sh = field_shapes(nx, ny, nz)
    vb = {"vx": np.zeros(sh["vx"]), "vy": np.zeros(sh["vy"]), "vz": np.zeros(sh["vz"])}
    txx, tyy, tzz = bc * so_bar["sxx"], bc * so_bar["syy"], bc * so_bar["szz"]
    tr = (txx + tyy + tzz) / 3.0
    # normal strains: exx = (Vx_{i+1} - Vx_i)/dx - div/3, and likewise
    vb["vx"][:, :, 1:] += (txx - tr) / dx
    vb["vx"][:, :, :-1] -= (txx - tr) / dx
    vb["vy"][:, 1:, :] += (tyy - tr) / dy
    vb["vy"][:, :-1, :] -= (tyy - tr) / dy
    vb["vz"][1:] += (tzz - tr) / dz
    vb["vz"][:-1] -= (tzz - tr) / dz
    # shear strains on interior edges: exy = 1/2 ((Vx_j - Vx_{j-1})/dy + (Vy_i - Vy_{i-1})/dx)
    txy = co["xy"][1] * so_bar["sxy"][:, 1:-1, 1:-1]
    vb["vx"][:, 1:, 1:-1] += 0.5 * txy / dy
    vb["vx"][:, :-1, 1:-1] -= 0.5 * txy / dy
    vb["vy"][:, 1:-1, 1:] += 0.5 * txy / dx
    vb["vy"][:, 1:-1, :-1] -= 0.5 * txy / dx
    txz = co["xz"][1] * so_bar["sxz"][1:-1, :, 1:-1]
    vb["vx"][1:, :, 1:-1] += 0.5 * txz / dz
    vb["vx"][:-1, :, 1:-1] -= 0.5 * txz / dz
    vb["vz"][1:-1, :, 1:] += 0.5 * txz / dx
    vb["vz"][1:-1, :, :-1] -= 0.5 * txz / dx
    tyz = co["yz"][1] * so_bar["syz"][1:-1, 1:-1, :]
    vb["vy"][1:, 1:-1, :] += 0.5 * tyz / dz
    vb["vy"][:-1, 1:-1, :] -= 0.5 * tyz / dz
    vb["vz"][1:-1, 1:, :] += 0.5 * tyz / dy
    vb["vz"][1:-1, :-1, :] -= 0.5 * tyz / dy
    # boundary faces are fixed (zero normal velocity): no adjoint there
    vb["vx"][:, :, 0] = vb["vx"][:, :, -1] = 0.0
    vb["vy"][:, 0, :] = vb["vy"][:, -1, :] = 0.0
    vb["vz"][0] = vb["vz"][-1] = 0.0
    prev = {}
    for k, key in (("sxx", "c"), ("syy", "c"), ("szz", "c"), ("sxy", "xy"), ("sxz", "xz"), ("syz", "yz")):
        a = co[key][0]
        out = np.zeros_like(so_bar[k])
        if key == "c":
            out[...] = a * so_bar[k]
        elif key == "xy":
            out[:, 1:-1, 1:-1] = a * so_bar[k][:, 1:-1, 1:-1]
        elif key == "xz":
            out[1:-1, :, 1:-1] = a * so_bar[k][1:-1, :, 1:-1]
        else:
            out[1:-1, 1:-1, :] = a * so_bar[k][1:-1, 1:-1, :]
        prev[k] = out
    return vb, prev


def run_forward(phys, nx, ny, nz, phi, logk0, n_steps, n_picard, rtol, max_iter=400000, record=True):
    """Picard run from the initial state; returns (oracle, tape).  tape[n][p]
    holds the stage's incoming ln(1-phi), its coefficients and its solution."""
    if phys.powerlaw or phys.dpcap:
        raise ValueError("the run adjoint needs the Newtonian viscosity law")
    o = Oracle(phys, nx, ny, nz, phi, np.exp(logk0))
    tape = []
    for _ in range(n_steps):
        o.begin_step()
        stages = []
        for _ in range(n_picard):
            o.refresh(1.0, 1.0)
            rec = {k: o.f[k].copy() for k in ("lp", "kc", "eta", "mus", "mn")} if record else None
            o.solve_linear(rtol, max_iter)
            if record:
                for k in ("vx", "vy", "vz", "pt", "pf"):
                    rec[k] = o.f[k].copy()
                stages.append(rec)
            o.porosity_step()
        tape.append(stages)
        o.end_step()
    return o, tape


def run_misfit(phys, nx, ny, nz, phi, logk0, sensors, d_obs, n_steps, n_picard, rtol, max_iter=400000):
    o, _ = run_forward(phys, nx, ny, nz, phi, logk0, n_steps, n_picard, rtol, max_iter, record=False)
    return misfit(o.f["pf"], sensors, d_obs)[0]


def run_adjoint(phys, nx, ny, nz, phi, logk0, sensors, d_obs, n_steps, n_picard, rtol,
                adj_rtol=None, max_iter=400000):
    """J and dJ/d(ln k0) (cells) of a Picard run of n_steps x n_picard stages."""
    adj_rtol = rtol if adj_rtol is None else adj_rtol
    o, tape = run_forward(phys, nx, ny, nz, phi, logk0, n_steps, n_picard, rtol, max_iter)
    J, g = misfit(o.f["pf"], sensors, d_obs)
    sh = field_shapes(nx, ny, nz)
    xbar = _zero_rhs(o)
    xbar["pf"] = g
    Lbar = np.zeros(sh["cell"])
    so_bar = {k: np.zeros(sh[kind]) for k, kind in (("sxx", "cell"), ("syy", "cell"), ("szz", "cell"),
                                                    ("sxy", "sxy"), ("sxz", "sxz"), ("syz", "syz"))}
    m_bar = np.zeros(sh["cell"])
    for n in reversed(range(n_steps)):
        acc = {"pto": np.zeros(sh["cell"]), "pfo": np.zeros(sh["cell"]), "lo": np.zeros(sh["cell"]),
               "fo": {k: np.zeros(sh[k]) for k in ("vx", "vy", "vz")}}
        mus = tape[n][0]["mus"]
        for p in reversed(range(n_picard)):
            rec = tape[n][p]
            eta_bar, s_bar_phi = porosity_step_adjoint(o, rec, Lbar, xbar, acc)
            lam, _, _ = solve_transposed(o, xbar, adj_rtol, max_iter, coef=rec)
            K_bar, chi_bar, s_bar_f = stage_parameter_adjoint(o, rec, lam, acc)
            Lbar, mb = coefficient_adjoint(o, rec, K_bar, eta_bar, s_bar_phi + s_bar_f, chi_bar)
            m_bar += mb
            xbar = _zero_rhs(o)       # x of the previous stage only seeds the PT solve
        # begin_step of step n: Lo = L, Pto = Pt, Pfo = Pf of the end of step n-1
        Lbar = Lbar + acc["lo"]
        xbar["pt"] += acc["pto"]
        xbar["pf"] += acc["pfo"]
        d = history_divergence_adjoint(o, acc["fo"], mus)
        for k in so_bar:
            so_bar[k] += d[k]
        if n >= 1:
            vb, so_bar = history_update_adjoint(o, so_bar, mus)
            for k in ("vx", "vy", "vz"):
                xbar[k] += vb[k]
    return J, m_bar
