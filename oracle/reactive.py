"""FP64 CPU reference of the reactive porosity-wave solver (thesis article 3).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU path never does, and the two share no
code (the seeded initial state comes from ``paper_2207_08716_amd.inputs``).

The arithmetic is in ``reactive.c``.  This module holds the state as numpy
arrays and runs the schedule of the appendix reactive script: per physical
step, the old values, then pseudo-transient iterations, the pseudo step
refreshed before iterations 1, nup+1, ..., the stopping quantity (the largest
one-iteration change of phi, Pf/10 and Xs) taken after iterations nup,
2 nup, ..., until it falls below eps or at iter_max.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import OracleDiverged, _load, _ptr


class _RwParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("phi0", C.c_double), ("k_muf0", C.c_double), ("eta", C.c_double),
                ("rho_f", C.c_double), ("rho_s", C.c_double), ("g", C.c_double),
                ("beta_d", C.c_double), ("beta_s", C.c_double), ("beta_f", C.c_double),
                ("tau", C.c_double), ("beta_x", C.c_double), ("delta_x", C.c_double), ("xs_max", C.c_double),
                ("dt", C.c_double), ("c_pf", C.c_double), ("phi_min", C.c_double), ("phi_max", C.c_double)]


_FIELDS = ("xs", "pf", "phi", "dpfdt", "xs_old", "pf_old", "phi_old")


class _RwState(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in _FIELDS]


def _lib():
    lib = _load()
    if not hasattr(lib, "_rw_ready"):
        P = C.POINTER
        lib.rw_create.restype = C.c_void_p
        lib.rw_create.argtypes = [P(_RwParams)]
        lib.rw_destroy.argtypes = [C.c_void_p]
        lib.rw_dtau.restype = C.c_double
        lib.rw_dtau.argtypes = [C.c_void_p, P(_RwState)]
        lib.rw_iteration.argtypes = [C.c_void_p, P(_RwState), C.c_double, P(C.c_double)]
        lib.rw_begin_step.argtypes = [C.c_void_p, P(_RwState)]
        lib._rw_ready = True
    return lib


class ReactiveOracle:
    """State and schedule of one reactive porosity-wave run.

    phys: paper_2207_08716_amd.inputs.WavePhysics (or any object with its
    fields); phi: initial porosity (nz, ny, nx); Xs starts at xs_max/2, Pf
    and dPf/dt at zero."""

    def __init__(self, phys, nx, ny, nz, phi, xs=None):
        self.phys = phys
        self.nx, self.ny, self.nz = nx, ny, nz
        self.lib = _lib()
        p = _RwParams()
        p.nx, p.ny, p.nz = nx, ny, nz
        for name, _ in _RwParams._fields_[3:]:
            setattr(p, name, float(getattr(phys, name)))
        self._params = p
        self.ctx = self.lib.rw_create(C.byref(p))
        if not self.ctx:
            raise ValueError("reactive oracle: bad grid")
        shape = (nz, ny, nx)
        self.f = {n: np.zeros(shape) for n in _FIELDS}
        self.f["phi"][...] = np.asarray(phi, dtype=np.float64)
        self.f["xs"][...] = 0.5 * phys.xs_max if xs is None else xs
        self._st = _RwState(*[_ptr(self.f[n]) for n in _FIELDS])
        self.iter = 0
        self.dtau = None
        self.last_err = None

    def __del__(self):
        try:
            if self.ctx:
                self.lib.rw_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def begin_step(self):
        self.lib.rw_begin_step(self.ctx, C.byref(self._st))
        self.iter = 0

    def iterate(self, n, dtau=None):
        """n PT iterations continuing the step's count: the pseudo step
        before iterations with iter % nup == 1, the error after iterations
        with iter % nup == 0 (returned, last one).  dtau, if given, replaces
        the pseudo step the state would give (a window of a larger grid
        takes the full grid's)."""
        nup = self.phys.nup
        for _ in range(n):
            it = self.iter + 1
            if (it - 1) % nup == 0:
                self.dtau = float(self.lib.rw_dtau(self.ctx, C.byref(self._st))) if dtau is None else float(dtau)
            err = C.c_double()
            want = it % nup == 0
            self.lib.rw_iteration(self.ctx, C.byref(self._st), self.dtau, C.byref(err) if want else None)
            self.iter = it
            if want:
                if not np.isfinite(err.value):
                    raise OracleDiverged(f"reactive: non-finite error at iteration {it}")
                self.last_err = err.value
        return self.last_err

    def solve_step(self, eps, iter_max):
        """Iterate until the error falls below eps (checked every nup) or
        iter_max; returns (iterations, error)."""
        nup = self.phys.nup
        err = np.inf
        while self.iter < iter_max:
            err = self.iterate(min(nup, iter_max - self.iter))
            if self.iter % nup == 0 and err < eps:
                break
        return self.iter, err
