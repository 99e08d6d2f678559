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

from . import Oracle


def misfit(pf: np.ndarray, sensors: np.ndarray, d_obs: np.ndarray):
    """J and dJ/dPf (a cell field) for sensor cells given as linear indices."""
    v = pf.ravel()[sensors]
    r = v - d_obs
    g = np.zeros(pf.size)
    g[sensors] = r
    return 0.5 * float(np.dot(r, r)), g.reshape(pf.shape)


def solve_adjoint(fwd: Oracle, g_pf: np.ndarray, rtol: float = 1e-12, max_iter: int = 400000):
    """lambda = (lam_vx, lam_vy, lam_vz, lam_pt, lam_pf) with J_F lambda = (0, 0, g)
    for the stage whose frozen coefficients and porosity are those of `fwd`."""
    ph = fwd.phys.replace(rhofg=0.0, rhosg=0.0)
    a = Oracle(ph, fwd.nx, fwd.ny, fwd.nz, 1.0 - np.exp(fwd.f["lp"]), None)
    for name in ("lp", "kc", "eta", "mus", "mn"):
        a.f[name][...] = fwd.f[name]
    ph0 = fwd.phys
    pfo = g_pf * ph0.dt / (ph0.beta_d * ph0.alpha * (1.0 / ph0.B - ph0.alpha))
    a.f["pfo"][...] = pfo
    a.f["pto"][...] = ph0.alpha * pfo
    a.refreshed = True          # coefficients are given, never refreshed here
    a.ref = None
    it, rho = a.solve_linear(rtol, max_iter)
    return {k: a.f[k].copy() for k in ("vx", "vy", "vz", "pt", "pf")}, it, rho


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
