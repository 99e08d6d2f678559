"""FP64 CPU reference ("oracle") of the pseudo-transient two-phase solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product path (the HIP library
and its Python binding) never imports or calls it, and the two share no code:
the only thing both sides consume is the seeded initial state from
``paper_2207_08716_amd.inputs``, passed in as plain arrays.

The arithmetic lives in ``oracle.c`` (plain C, FP64, no FMA contraction,
OpenMP over z only).  This module allocates the state as numpy arrays, passes
pointers through ctypes and runs the two schedules of the method:

* thesis schedule (article 1; appendix two-phase script): every PT iteration
  updates velocities, pressures and porosity; the lagged coefficients are
  refreshed with log relaxation before iterations 1, nup+1, 2 nup+1, ...; the
  residual norms and the one-iteration change are taken after iterations
  nup, 2 nup, ...;
* Picard schedule: per physical step, P stages; each refreshes the
  coefficients without relaxation, solves the resulting linear system for
  (V, Pt, Pf) by PT iterations with porosity frozen, down to a relative
  residual rtol, and then advances ln(1-phi) by one step of eq (22).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")
SOURCES = (SRC_PATH, os.path.join(_HERE, "reactive.c"))

NORM_NAMES = ("f", "rpt", "rpf", "dL", "dPt", "dPf", "dVz", "dV")

# Alternative readings of the iteration (oracle.c OR_V_*); 0 = the readings
# the solver implements.  They change the pseudo-time path, not the solution.
V_BETAN_UPDATED = 1   # beta_n r_Pt in the stresses taken at the updated Pt'
V_DTV_PRINTED = 2     # velocity pseudo-step with (1+beta_n) as printed
V_DTPF_CELL = 4       # fluid-pressure pseudo-step from the cell's own k/mu_f


class OracleDiverged(FloatingPointError):
    """A residual norm of the oracle is not finite."""


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", tmp, *SOURCES, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("phi0", C.c_double), ("kmuf0", C.c_double), ("eta0", C.c_double),
                ("mu0", C.c_double), ("cmu", C.c_double), ("rhofg", C.c_double),
                ("rhosg", C.c_double), ("beta_phi", C.c_double), ("beta_d", C.c_double),
                ("alpha", C.c_double), ("B", C.c_double), ("G", C.c_double),
                ("R0", C.c_double), ("n_pow", C.c_double), ("tau0", C.c_double),
                ("coh", C.c_double), ("fric_deg", C.c_double), ("tau_y_min", C.c_double),
                ("dt", C.c_double), ("dtS", C.c_double), ("beta_n", C.c_double),
                ("rho_i", C.c_double), ("c_v", C.c_double), ("c_pf", C.c_double),
                ("damp_c", C.c_double),
                ("powerlaw", C.c_int32), ("dpcap", C.c_int32), ("mech_off", C.c_int32),
                ("k0field", C.c_int32), ("ngx", C.c_int32), ("ngy", C.c_int32), ("ngz", C.c_int32),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("variant", C.c_int32), ("shear_bg", C.c_double)]


_STATE_FIELDS = ("vx", "vy", "vz", "pt", "pf", "lp", "rx", "ry", "rz", "pto", "pfo",
                 "lpo", "sxx", "syy", "szz", "sxy", "sxz", "syz", "mn", "k0", "kc",
                 "eta", "mus")
_SOURCE_FIELDS = ("fsx", "fsy", "fsz")


class _State(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in _STATE_FIELDS + _SOURCE_FIELDS]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(os.path.getmtime(f) for f in SOURCES):
            build()
        lib = C.CDLL(LIB_PATH)
        P = C.POINTER
        lib.or_create.restype = C.c_void_p
        lib.or_create.argtypes = [P(_Params)]
        lib.or_destroy.argtypes = [C.c_void_p]
        lib.or_iteration.argtypes = [C.c_void_p, P(_State), C.c_int, P(C.c_double)]
        lib.or_residual.argtypes = [C.c_void_p, P(_State)] + [P(C.c_double)] * 5
        lib.or_porosity_step.argtypes = [C.c_void_p, P(_State)]
        lib.or_begin_step.argtypes = [C.c_void_p, P(_State), C.c_int]
        lib.or_refresh.argtypes = [C.c_void_p, P(_State), C.c_int, C.c_double, C.c_double]
        lib.or_tau_ii.argtypes = [C.c_void_p, P(_State), P(C.c_double)]
        lib.or_last_stresses.argtypes = [C.c_void_p] + [P(C.c_double)] * 6
        lib.or_last_fluxes.argtypes = [C.c_void_p] + [P(C.c_double)] * 3
        lib.or_num_threads.restype = C.c_int
        lib.or_set_dts.argtypes = [C.c_void_p, C.c_double]
        lib.or_max_mus.argtypes = [C.c_void_p, P(_State)]
        lib.or_max_mus.restype = C.c_double
        lib.or_set_num_threads.argtypes = [C.c_int]
        lib.or_heat1d_step.restype = C.c_int
        lib.or_heat1d_step.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                                       C.c_double, P(C.c_double), P(C.c_double), C.c_int]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def field_shapes(nx, ny, nz):
    """(z, y, x) shapes of every staggered field."""
    return {
        "cell": (nz, ny, nx),
        "vx": (nz, ny, nx + 1), "vy": (nz, ny + 1, nx), "vz": (nz + 1, ny, nx),
        "sxy": (nz, ny + 1, nx + 1), "sxz": (nz + 1, ny, nx + 1), "syz": (nz + 1, ny + 1, nx),
    }


_SHAPE_KIND = {"vx": "vx", "vy": "vy", "vz": "vz", "rx": "vx", "ry": "vy", "rz": "vz",
               "sxy": "sxy", "sxz": "sxz", "syz": "syz"}


class Oracle:
    """FP64 CPU solver state and schedules.

    phys: paper_2207_08716_amd.inputs.Physics (any object with its fields).
    phi:  initial porosity, (nz, ny, nx).  k0: per-cell k0/mu_f or None.
    """

    def __init__(self, phys, nx, ny, nz, phi, k0=None, global_counts=None, variant=0):
        """global_counts: (nx, ny, nz) of the full grid on the domain of phys
        when these arrays are a window of it (the spacing, the damping and
        the Pt pseudo-step are the full grid's).  variant: V_* bits selecting
        alternative readings of the iteration (0: the solver's)."""
        self.phys = phys
        self.nx, self.ny, self.nz = nx, ny, nz
        self.lib = _load()
        p = _Params()
        p.nx, p.ny, p.nz = nx, ny, nz
        for name, _ in _Params._fields_[3:-12]:
            setattr(p, name, float(getattr(phys, name)))
        if global_counts is not None:
            # a window of a (gx, gy, gz) grid on the full domain of phys
            gx, gy, gz = (int(v) for v in global_counts)
            p.ngx, p.ngy, p.ngz = gx, gy, gz
            p.hx, p.hy, p.hz = phys.lx / gx, phys.ly / gy, phys.lz / gz
        p.powerlaw = int(bool(phys.powerlaw))
        p.dpcap = int(bool(phys.dpcap))
        p.mech_off = int(bool(phys.mech_off))
        p.k0field = int(k0 is not None)
        p.variant = int(variant)
        p.shear_bg = float(getattr(phys, "shear_bg", 0.0))
        self._params = p
        self.ctx = self.lib.or_create(C.byref(p))
        if not self.ctx:
            raise ValueError("oracle: bad grid")
        shapes = field_shapes(nx, ny, nz)
        self.f = {}
        for name in _STATE_FIELDS:
            kind = _SHAPE_KIND.get(name, "cell")
            self.f[name] = np.zeros(shapes[kind], dtype=np.float64)
        phi = np.asarray(phi, dtype=np.float64)
        assert phi.shape == shapes["cell"]
        self.f["lp"][...] = np.log(1.0 - phi)
        self.f["lpo"][...] = self.f["lp"]
        self.f["mn"][...] = phys.mu0
        if k0 is not None:
            self.f["k0"][...] = k0
        # coefficients before the first refresh (overwritten by it)
        self.f["eta"][...] = 1.0
        self.f["mus"][...] = phys.mu0 * phys.phi0 * phys.cmu
        self.f["kc"][...] = phys.kmuf0
        self.source = None     # optional momentum source (adjoint solves only)
        self._bind()
        self.refreshed = False
        self.step_index = 0
        # stress-history step rule of the script (per-step block): the
        # accumulated time since the last history update starts at dt
        self.dt_cum = float(phys.dt)
        self.dts = float(phys.dtS)
        self.iter = 0          # iteration counter within the current step
        self.total_iters = 0
        self.history = []      # norms at each check

    def _bind(self):
        src = [None] * 3 if self.source is None else [_ptr(a) for a in self.source]
        self._st = _State(*([_ptr(self.f[n]) for n in _STATE_FIELDS] + src))

    def set_momentum_source(self, fx, fy, fz):
        """Additive momentum source on the interior faces (None: remove).  Not
        part of the method: the adjoint uses it to impose a right-hand side
        on the momentum rows of a transposed solve."""
        if fx is None:
            self.source = None
        else:
            sh = field_shapes(self.nx, self.ny, self.nz)
            self.source = tuple(np.ascontiguousarray(a, dtype=np.float64).copy()
                                for a in (fx, fy, fz))
            assert [a.shape for a in self.source] == [sh["vx"], sh["vy"], sh["vz"]]
        self._bind()

    def __del__(self):
        try:
            if self.ctx:
                self.lib.or_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # ---- primitives ---------------------------------------------------------
    def begin_step(self):
        """Old values; stress history from the current state from step 2 on.

        With the stress-history step rule (phys.dts_rule, the script's
        per-step block): dtS = max(mu_s) / (G xi_w) each step; the history is
        renewed (with the stresses of the previous dtS) when the time
        accumulated since the last renewal reaches the new dtS, and that
        accumulation restarts; the first step keeps the zero history."""
        ph = self.phys
        if getattr(ph, "dts_rule", False):
            dts_new = float(self.lib.or_max_mus(self.ctx, C.byref(self._st))) / (ph.G * ph.xsi_w)
            renew = self.step_index >= 1 and self.dt_cum >= dts_new
            self.lib.or_begin_step(self.ctx, C.byref(self._st), int(renew))
            if renew or self.step_index == 0:
                self.dt_cum = 0.0
            self.dts = dts_new
            self.lib.or_set_dts(self.ctx, dts_new)
            self.history_renewed = renew
        else:
            self.lib.or_begin_step(self.ctx, C.byref(self._st), int(self.step_index >= 1))
            self.history_renewed = self.step_index >= 1
        self.iter = 0
        self.ref = None        # residual reference of the step, set by its first solve

    def end_step(self):
        self.step_index += 1
        self.dt_cum += float(self.phys.dt)

    def refresh(self, r_eta=None, r_mu=None):
        ph = self.phys
        r_eta = ph.r_eta if r_eta is None else r_eta
        r_mu = ph.r_mu if r_mu is None else r_mu
        self.lib.or_refresh(self.ctx, C.byref(self._st), int(not self.refreshed),
                            float(r_eta), float(r_mu))
        self.refreshed = True

    def iteration(self, update_lp=True, norms=False):
        out = np.zeros(8) if norms else None
        self.lib.or_iteration(self.ctx, C.byref(self._st), int(update_lp), _ptr(out))
        self.iter += 1
        self.total_iters += 1
        return None if out is None else dict(zip(NORM_NAMES, out.tolist()))

    def residual(self):
        """(fx, fy, fz, r_Pt, r_Pf) at the current state and coefficients."""
        sh = field_shapes(self.nx, self.ny, self.nz)
        out = [np.zeros(sh["vx"]), np.zeros(sh["vy"]), np.zeros(sh["vz"]),
               np.zeros(sh["cell"]), np.zeros(sh["cell"])]
        self.lib.or_residual(self.ctx, C.byref(self._st), *[_ptr(a) for a in out])
        return out

    def porosity_step(self):
        self.lib.or_porosity_step(self.ctx, C.byref(self._st))

    def tau_ii(self):
        out = np.zeros((self.nz, self.ny, self.nx))
        self.lib.or_tau_ii(self.ctx, C.byref(self._st), _ptr(out))
        return out

    def last_stresses(self):
        sh = field_shapes(self.nx, self.ny, self.nz)
        out = [np.zeros(sh["cell"]) for _ in range(3)] + [np.zeros(sh["sxy"]), np.zeros(sh["sxz"]), np.zeros(sh["syz"])]
        self.lib.or_last_stresses(self.ctx, *[_ptr(a) for a in out])
        return out

    def last_fluxes(self):
        sh = field_shapes(self.nx, self.ny, self.nz)
        out = [np.zeros(sh["vx"]), np.zeros(sh["vy"]), np.zeros(sh["vz"])]
        self.lib.or_last_fluxes(self.ctx, *[_ptr(a) for a in out])
        return out

    # ---- thesis schedule ----------------------------------------------------
    def iterate(self, n):
        """n PT iterations of the thesis schedule, continuing the step's
        iteration count: refresh (with relaxation, none at the first refresh
        of the run) before iterations with (iter-1) % nup == 0; norms after
        iterations with iter % nup == 0 (stored in self.history)."""
        nup = self.phys.nup
        last = None
        for _ in range(n):
            it = self.iter + 1
            if (it - 1) % nup == 0:
                self.refresh()
            nm = self.iteration(update_lp=True, norms=(it % nup == 0))
            if nm is not None:
                _check_finite(nm, it)
                nm["iter"] = it
                self.history.append(nm)
                last = nm
        return last

    # ---- Picard schedule ----------------------------------------------------
    def solve_linear(self, rtol, max_iter=200000):
        """PT iterations with porosity and coefficients frozen until
        rho = max(g_V/g_V0, g_P/g_P0) <= rtol, checked every nup iterations;
        g_V = max|f|, g_P = max(|r_Pt|, |r_Pf|); 0 = the residual at the first
        iteration of the step's first solve (kept for its later Picard
        stages, whose own initial residuals are already small)."""
        nup = self.phys.nup
        it = 0
        rho = np.inf
        if not hasattr(self, "ref"):
            self.ref = None
        while it < max_iter:
            it += 1
            want = (it == 1 and self.ref is None) or (it % nup == 0)
            nm = self.iteration(update_lp=False, norms=want)
            if nm is None:
                continue
            _check_finite(nm, it)
            gv, gp = nm["f"], max(nm["rpt"], nm["rpf"])
            if self.ref is None:
                self.ref = (gv, gp)
            rho = rel_residual(gv, gp, self.ref)
            if it % nup == 0 and rho <= rtol:
                break
        return it, rho

    def picard_step(self, n_picard, rtol, max_iter=200000):
        """One physical step of the Picard schedule; returns iteration counts."""
        self.begin_step()
        counts = []
        for _ in range(n_picard):
            self.refresh(r_eta=1.0, r_mu=1.0)
            it, rho = self.solve_linear(rtol, max_iter)
            counts.append((it, rho))
            self.porosity_step()
        self.end_step()
        return counts

    # ---- views --------------------------------------------------------------
    def phi(self):
        return 1.0 - np.exp(self.f["lp"])


def _check_finite(nm, it):
    bad = [k for k in NORM_NAMES if not np.isfinite(nm[k])]
    if bad:
        raise OracleDiverged(f"non-finite norms {bad} at iteration {it}")


def rel_residual(gv, gp, g0):
    """rho = max over groups with a nonzero initial norm of g/g0.  Raises
    OracleDiverged if any norm is not finite (Python's max would drop a NaN
    and report a diverged solve as converged)."""
    if not all(np.isfinite(v) for v in (gv, gp, g0[0], g0[1])):
        raise OracleDiverged(f"non-finite residual: g_V {gv}, g_P {gp}, reference {g0}")
    r = 0.0
    if g0[0] > 0:
        r = max(r, gv / g0[0])
    if g0[1] > 0:
        r = max(r, gp / g0[1])
    return r


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's following OpenMP loops (timing only)."""
    _load().or_set_num_threads(int(n))


def heat1d_step(Ut, U0, dx, dt, lam_rho_cp, eps, max_iter=10_000_000):
    """One implicit time step of the 1D PT heat example (article 1, Fig. 2)."""
    lib = _load()
    Ut = np.ascontiguousarray(Ut, dtype=np.float64)
    U = np.array(U0, dtype=np.float64, copy=True)
    it = lib.or_heat1d_step(len(U), dx, dt, lam_rho_cp, eps, _ptr(Ut), _ptr(U), max_iter)
    return U, it
