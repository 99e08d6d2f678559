"""Python handle over the HIP solver: torch owns the device buffers and the
stream, the C library (libptporo.so) does every step of the computation.

Methods map one-to-one onto the C entry points; this module only allocates
buffers, passes pointers and converts fields between the padded device layout
and compact (z, y, x) numpy arrays for inspection.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import abi


# Stride skew of the mixed workspace's FP32 boxes (floats), as in ptporo.h.
MIXED_BOX_SKEW = 64
# Skew between consecutive field buffers of one grid (doubles): buffers a
# power of two apart (1 GiB at 511^3) put the sweep's 27 streams on the same
# memory channels at the same moment; one skewed allocation sweeps ~5 %
# faster at 511^3 than separate buffers (thesis sweep 6.70 -> 6.36 ms).
FIELD_SKEW = 32


def field_extent(name, nx, ny, nz):
    """(z, y, x) extent of a field inside its padded box."""
    if name in ("vx", "rx", "fox"):
        return (nz, ny, nx + 1)
    if name in ("vy", "ry", "foy"):
        return (nz, ny + 1, nx)
    if name in ("vz", "rz", "foz"):
        return (nz + 1, ny, nx)
    if name == "sxy":
        return (nz, ny + 1, nx + 1)
    if name == "sxz":
        return (nz + 1, ny, nx + 1)
    if name == "syz":
        return (nz + 1, ny + 1, nx)
    return (nz, ny, nx)


def _check(lib, h, st, what):
    if st < 0:
        msg = lib.pt_last_error(h).decode() if h else ""
        raise abi.PTError(st, f"{what}: {msg}")
    return st


class Grid:
    """Solver state on one GPU for an nx x ny x nz cell grid.

    phys: paper_2207_08716_amd.inputs.Physics.  k0field: bind a per-cell
    k0/mu_f field.  The row pitch is padded to a multiple of 32 elements.
    """

    def __init__(self, phys, nx, ny, nz, k0field=False, device="cuda", pitch=None, stream=None):
        self.lib = abi.load()
        self.phys = phys
        self.nx, self.ny, self.nz = nx, ny, nz
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on the GPU only")
        self.pitch = pitch or ((nx + 1 + 31) // 32) * 32
        self.k0field = bool(k0field)
        self._params = abi.params_from(phys, self.k0field)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = None
        self._create_handle()
        box = (nz + 1, ny + 1, self.pitch)
        assert self.lib.pt_field_elems(self.h) == box[0] * box[1] * box[2]
        self.buf = {}
        nel = box[0] * box[1] * box[2]
        names = [(fid, name) for fid, name in enumerate(abi.FIELDS) if name != "k0" or self.k0field]
        count = sum(2 if fid < abi.NPING else 1 for fid, _ in names)
        stride = nel + FIELD_SKEW
        with torch.cuda.stream(self.stream):
            # every field from one allocation, consecutive buffers one box and
            # 256 bytes apart (base 256-byte aligned)
            self.arena = torch.zeros(count * stride + 32, dtype=torch.float64, device=self.device)
            base = (-self.arena.data_ptr() // 8) % 32
            k = 0
            for fid, name in names:
                self.buf[name] = []
                for _ in range(2 if fid < abi.NPING else 1):
                    off = base + k * stride
                    self.buf[name].append(self.arena[off:off + nel].view(box))
                    k += 1
            nbytes = C.c_size_t()
            _check(self.lib, self.h, self.lib.pt_workspace_size(self.h, C.byref(nbytes)), "workspace_size")
            self.ws = torch.zeros((nbytes.value + 7) // 8, dtype=torch.float64, device=self.device)
            self.ws_bytes = nbytes.value
        self._bind_all()

    def _create_handle(self):
        h = C.c_void_p()
        st = self.lib.pt_create(self.nx, self.ny, self.nz, self.pitch, C.byref(self._params), C.byref(h))
        if st != 0:
            raise abi.PTError(st, "pt_create rejected the grid or parameters")
        self.h = h
        _check(self.lib, h, self.lib.pt_set_stream(h, C.c_void_p(self.stream.cuda_stream)), "set_stream")

    def _bind_all(self):
        h = self.h
        for name, bufs in self.buf.items():
            fid = abi.FIELD_ID[name]
            for cp, t in enumerate(bufs):
                _check(self.lib, h, self.lib.pt_bind_field(h, fid, cp, C.c_void_p(t.data_ptr())), f"bind {name}")
        _check(self.lib, h, self.lib.pt_bind_workspace(h, C.c_void_p(self.ws.data_ptr()), self.ws_bytes), "bind ws")
        if getattr(self, "mws", None) is not None:
            _check(self.lib, h, self.lib.pt_bind_mixed_workspace(h, C.c_void_p(self.mws.data_ptr()),
                                                                 self.mws_bytes), "bind mixed")
        if getattr(self, "aws", None) is not None:
            _check(self.lib, h, self.lib.pt_bind_adjoint_workspace(h, C.c_void_p(self.aws.data_ptr()),
                                                                   self.aws_bytes, int(self.aws_sensors)),
                   "bind adjoint")
        if getattr(self, "gws", None) is not None:
            _check(self.lib, h, self.lib.pt_bind_mg_workspace(h, C.byref(self.gws_params),
                                                              C.c_void_p(self.gws.data_ptr()),
                                                              self.gws.numel() * 8), "bind mg")

    # ---- resuming on a new handle ----------------------------------------------
    def counters(self) -> abi.Counters:
        c = abi.Counters()
        _check(self.lib, self.h, self.lib.pt_get_counters(self.h, C.byref(c)), "get_counters")
        return c

    def set_counters(self, c: abi.Counters):
        _check(self.lib, self.h, self.lib.pt_set_counters(self.h, C.byref(c)), "set_counters")

    def recreate_handle(self):
        """Destroy the C handle and create a new one on the same buffers,
        carrying the counters over (the run continues bit for bit)."""
        c = self.counters()
        self.lib.pt_destroy(self.h)
        self.h = None
        self._create_handle()
        self._bind_all()
        self.set_counters(c)

    def close(self):
        if getattr(self, "h", None):
            self.lib.pt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state access --------------------------------------------------------
    def tensor(self, name):
        """Device tensor (padded box) holding the present value of a field
        (the damped residual is stored first, see pt_sync_damped_residual)."""
        fid = abi.FIELD_ID[name]
        if name in ("rx", "ry", "rz"):
            _check(self.lib, self.h, self.lib.pt_sync_damped_residual(self.h), "sync damped residual")
        cp = C.c_int32()
        _check(self.lib, self.h, self.lib.pt_current(self.h, fid, C.byref(cp)), "current")
        return self.buf[name][cp.value]

    def view(self, name):
        """Device view of the field's extent inside its padded box."""
        ez, ey, ex = field_extent(name, self.nx, self.ny, self.nz)
        return self.tensor(name)[:ez, :ey, :ex]

    def get(self, name) -> np.ndarray:
        with torch.cuda.stream(self.stream):
            out = self.view(name).cpu().numpy().copy()
        return out

    def set(self, name, value):
        """Write a field (numpy array of the field's extent, or a scalar) into
        the present copy."""
        with torch.cuda.stream(self.stream):
            v = self.view(name)
            if np.isscalar(value):
                v.fill_(float(value))
            else:
                a = np.ascontiguousarray(value, dtype=np.float64)
                assert a.shape == tuple(v.shape), (name, a.shape, tuple(v.shape))
                v.copy_(torch.from_numpy(a).to(self.device, non_blocking=False))

    def load_initial(self, phi, k0=None):
        """Initial state of every workload (pt_reset_state, pt_set_porosity):
        V = R = 0, pressures 0, stress history 0, ln(1-phi) from phi, Mn = mu0;
        coefficients take their background values until the first refresh."""
        if self.k0field:
            if k0 is None:
                raise ValueError("k0 field expected")
            self.set("k0", k0)
        elif k0 is not None:
            raise ValueError("grid created without a k0 field")
        self.reset_state(phi)

    # ---- solver entry points --------------------------------------------------
    def begin_step(self, update_history=False):
        _check(self.lib, self.h, self.lib.pt_begin_step(self.h, int(bool(update_history))), "begin_step")

    def refresh(self, r_eta=None, r_mu=None):
        r_eta = self.phys.r_eta if r_eta is None else r_eta
        r_mu = self.phys.r_mu if r_mu is None else r_mu
        _check(self.lib, self.h, self.lib.pt_refresh(self.h, float(r_eta), float(r_mu)), "refresh")

    def iteration(self, update_lp=True, norms=False):
        _check(self.lib, self.h, self.lib.pt_iteration(self.h, int(bool(update_lp)), int(bool(norms))), "iteration")

    def iterate(self, n):
        _check(self.lib, self.h, self.lib.pt_iterate(self.h, int(n)), "iterate")

    def last_norms(self) -> dict:
        nm = abi.Norms()
        _check(self.lib, self.h, self.lib.pt_last_norms(self.h, C.byref(nm)), "last_norms")
        return {n: getattr(nm, n) for n, _ in abi.Norms._fields_}

    def solve_linear(self, rtol, max_iter=1_000_000):
        it = C.c_int64()
        rho = C.c_double()
        st = _check(self.lib, self.h, self.lib.pt_solve_linear(self.h, float(rtol), int(max_iter),
                                                                 C.byref(it), C.byref(rho)), "solve_linear")
        return it.value, rho.value, st == 0

    def solve_linear_static(self, rtol, max_iter=1_000_000):
        """pt_solve_linear_static: the same solve with the library's static
        device scratch in place of the workspace (allocates nothing)."""
        it = C.c_int64()
        rho = C.c_double()
        st = _check(self.lib, self.h, self.lib.pt_solve_linear_static(self.h, float(rtol), int(max_iter),
                                                                        C.byref(it), C.byref(rho)),
                    "solve_linear_static")
        return it.value, rho.value, st == 0

    def residual_reference(self):
        gv = C.c_double()
        gp = C.c_double()
        _check(self.lib, self.h, self.lib.pt_residual_reference(self.h, C.byref(gv), C.byref(gp)), "reference")
        return (gv.value, gp.value) if gv.value >= 0 else None

    def set_residual_reference(self, ref):
        gv, gp = ref if ref is not None else (-1.0, -1.0)
        _check(self.lib, self.h, self.lib.pt_set_residual_reference(self.h, float(gv), float(gp)), "set reference")

    def porosity_step(self):
        _check(self.lib, self.h, self.lib.pt_porosity_step(self.h), "porosity_step")

    def picard_step(self, update_history, n_picard, rtol, max_iter=2_000_000, mixed=False, eta_in=1e-4,
                    solver=None):
        """One physical step of the Picard schedule (see pt_picard_step):
        returns (sweeps, rho, converged).  solver: "fp64", "mixed" or "mg"
        (default: "mixed" if mixed else "fp64"); for "mg", max_iter bounds
        the V-cycles of a stage and sweeps counts V-cycles."""
        solver = solver or ("mixed" if mixed else "fp64")
        code = {"fp64": abi.SOLVER_FP64, "mixed": abi.SOLVER_MIXED, "mg": abi.SOLVER_MG}[solver]
        if solver == "mixed":
            self.enable_mixed()
        elif solver == "mg" and getattr(self, "gws", None) is None:
            self.enable_mg()
        sweeps = C.c_int64()
        rho = C.c_double()
        st = _check(self.lib, self.h, self.lib.pt_picard_step(self.h, int(bool(update_history)), int(n_picard),
                                                               float(rtol), int(max_iter), code,
                                                               float(eta_in), C.byref(sweeps), C.byref(rho)),
                    "picard_step")
        return sweeps.value, rho.value, st == 0

    # ---- geometric multigrid ------------------------------------------------
    def enable_mg(self, **params):
        """Allocate and bind the multigrid workspace (see pt_mg_params; keyword
        arguments override its defaults).  Rebinds when the parameters change."""
        mp = abi.mg_params(**params)
        key = tuple(getattr(mp, n) for n, _ in abi.MgParams._fields_)
        if getattr(self, "gws", None) is not None and self.gws_key == key:
            return
        nbytes = C.c_size_t()
        _check(self.lib, self.h, self.lib.pt_mg_workspace_size(self.h, C.byref(mp), C.byref(nbytes)), "mg size")
        self.gws = None
        with torch.cuda.stream(self.stream):
            self.gws = torch.empty((nbytes.value + 7) // 8, dtype=torch.float64, device=self.device)
        _check(self.lib, self.h, self.lib.pt_bind_mg_workspace(self.h, C.byref(mp), C.c_void_p(self.gws.data_ptr()),
                                                               nbytes.value), "bind mg")
        self.gws_key = key
        self.gws_params = mp

    def mg_levels(self):
        """Cell counts (nx, ny, nz) of every grid of the bound hierarchy."""
        n = C.c_int32()
        counts = (C.c_int32 * (3 * abi.MG_MAX_LEVELS))()
        _check(self.lib, self.h, self.lib.pt_mg_levels(self.h, C.byref(n), counts), "mg levels")
        return [tuple(counts[3 * l:3 * l + 3]) for l in range(n.value)]

    def solve_mg(self, rtol, max_cycles=200, **params):
        """Multigrid solve of the present Picard stage (see pt_solve_mg):
        returns (cycles, rho, converged).  Keyword arguments rebind the
        workspace with those parameters; without them the bound hierarchy
        (or a default one) is used."""
        if params or getattr(self, "gws", None) is None:
            self.enable_mg(**params)
        cyc = C.c_int64()
        rho = C.c_double()
        st = _check(self.lib, self.h, self.lib.pt_solve_mg(self.h, float(rtol), int(max_cycles), C.byref(cyc),
                                                            C.byref(rho)), "solve_mg")
        return cyc.value, rho.value, st == 0

    # ---- mixed precision ----------------------------------------------------
    def enable_mixed(self):
        """Allocate and bind the FP32 workspace of the defect-correction solve."""
        if getattr(self, "mws", None) is not None:
            return
        nbytes = C.c_size_t()
        _check(self.lib, self.h, self.lib.pt_mixed_workspace_size(self.h, C.byref(nbytes)), "mixed size")
        with torch.cuda.stream(self.stream):
            self.mws = torch.zeros((nbytes.value + 3) // 4, dtype=torch.float32, device=self.device)
        self.mws_bytes = nbytes.value
        _check(self.lib, self.h, self.lib.pt_bind_mixed_workspace(self.h, C.c_void_p(self.mws.data_ptr()),
                                                                  nbytes.value), "bind mixed")

    def residual(self):
        """FP64 residual norms of the present state (see pt_residual)."""
        self.enable_mixed()
        _check(self.lib, self.h, self.lib.pt_residual(self.h), "residual")
        return self.last_norms()

    def residual_fields(self):
        """(fx, fy, fz, r_Pt, r_Pf) last written by residual(), as numpy."""
        box = (self.nz + 1) * (self.ny + 1) * self.pitch
        stride = box + MIXED_BOX_SKEW          # the workspace's box stride (ptporo.h)
        out = []
        for b, name in enumerate(("vx", "vy", "vz", "pt", "pf")):
            t = self.mws[(16 + b) * stride:(16 + b) * stride + box].view(self.nz + 1, self.ny + 1, self.pitch)
            ez, ey, ex = field_extent(name, self.nx, self.ny, self.nz)
            with torch.cuda.stream(self.stream):
                out.append(t[:ez, :ey, :ex].double().cpu().numpy())
        return out

    def solve_mixed(self, rtol, eta_in=1e-4, max_inner=1_000_000, max_outer=50):
        """Defect-correction solve of the present Picard stage (see pt_solve_mixed)."""
        self.enable_mixed()
        inner = C.c_int64()
        outer = C.c_int32()
        rho = C.c_double()
        st = _check(self.lib, self.h, self.lib.pt_solve_mixed(self.h, float(rtol), float(eta_in), int(max_inner),
                                                               int(max_outer), C.byref(inner), C.byref(outer),
                                                               C.byref(rho)), "solve_mixed")
        return inner.value, outer.value, rho.value, st == 0

    # ---- stage adjoint ------------------------------------------------------
    def enable_adjoint(self, max_sensors=64):
        """Allocate and bind the FP64 workspace of the stage adjoint."""
        if getattr(self, "aws", None) is not None and self.aws_sensors >= max_sensors:
            return
        nbytes = C.c_size_t()
        _check(self.lib, self.h, self.lib.pt_adjoint_workspace_size(self.h, int(max_sensors), C.byref(nbytes)),
               "adjoint size")
        with torch.cuda.stream(self.stream):
            self.aws = torch.zeros((nbytes.value + 7) // 8, dtype=torch.float64, device=self.device)
            self.grad_buf = torch.zeros(self.buf["pt"][0].shape, dtype=torch.float64, device=self.device)
        self.aws_bytes = nbytes.value
        _check(self.lib, self.h, self.lib.pt_bind_adjoint_workspace(self.h, C.c_void_p(self.aws.data_ptr()),
                                                                    nbytes.value, int(max_sensors)), "bind adjoint")
        self.aws_sensors = max_sensors

    def set_log_k0(self, logk0):
        """k0 <- exp(logk0): logk0 a (nz, ny, nx) array or device tensor."""
        if not self.k0field:
            raise ValueError("grid created without a k0 field")
        with torch.cuda.stream(self.stream):
            box = torch.zeros(self.buf["pt"][0].shape, dtype=torch.float64, device=self.device)
            t = torch.as_tensor(logk0, dtype=torch.float64, device=self.device)
            box[:self.nz, :self.ny, :self.nx].copy_(t)
        _check(self.lib, self.h, self.lib.pt_set_log_k0(self.h, C.c_void_p(box.data_ptr())), "set_log_k0")
        self.stream.synchronize()

    def misfit(self, sensors, d_obs) -> float:
        self.enable_adjoint(max(64, len(sensors)))
        s_arr = np.ascontiguousarray(sensors, dtype=np.int64)
        d_arr = np.ascontiguousarray(d_obs, dtype=np.float64)
        J = C.c_double()
        _check(self.lib, self.h, self.lib.pt_misfit(self.h, s_arr.ctypes.data_as(C.POINTER(C.c_int64)), len(s_arr),
                                                    d_arr.ctypes.data_as(C.POINTER(C.c_double)), C.byref(J)), "misfit")
        return J.value

    def adjoint_stage(self, sensors, d_obs, rtol=1e-12, max_iter=2_000_000):
        """J and dJ/d(ln k0) (device tensor view, cells) for the present
        linear Picard stage (see pt_adjoint_stage)."""
        self.enable_adjoint(max(64, len(sensors)))
        s_arr = np.ascontiguousarray(sensors, dtype=np.int64)
        d_arr = np.ascontiguousarray(d_obs, dtype=np.float64)
        J = C.c_double()
        it = C.c_int64()
        rho = C.c_double()
        st = _check(self.lib, self.h, self.lib.pt_adjoint_stage(
            self.h, s_arr.ctypes.data_as(C.POINTER(C.c_int64)), len(s_arr),
            d_arr.ctypes.data_as(C.POINTER(C.c_double)), float(rtol), int(max_iter),
            C.c_void_p(self.grad_buf.data_ptr()), C.byref(J), C.byref(it), C.byref(rho)), "adjoint_stage")
        return J.value, self.grad_buf[:self.nz, :self.ny, :self.nx], it.value, rho.value, st == 0

    def set_progress(self, fn):
        """fn(phase_name, step, stage, sweeps) after every stage of long calls
        (None: off)."""
        if fn is None:
            self._progress_cb = None
            _check(self.lib, self.h, self.lib.pt_set_progress(self.h, abi.PROGRESS_FN(), None), "progress")
            return

        def cb(_user, phase, step, stage, sweeps):
            fn(abi.PROGRESS_PHASE.get(phase, str(phase)), step, stage, sweeps)
        self._progress_cb = abi.PROGRESS_FN(cb)     # kept alive with the grid
        _check(self.lib, self.h, self.lib.pt_set_progress(self.h, self._progress_cb, None), "progress")

    def adjoint_run(self, sensors, d_obs, n_steps, n_picard, rtol=1e-12, adj_rtol=None, max_iter=2_000_000,
                    checkpoint=False, mixed=False):
        """Recorded Picard run of n_steps x n_picard stages from the present
        state and its adjoint (see pt_adjoint_run): returns J, dJ/d(ln k0)
        (device tensor view, cells), forward and transposed sweep counts.
        checkpoint: keep step checkpoints and recompute the stages in reverse;
        mixed: FP32 sweeps inside FP64 defect correction for every solve."""
        adj_rtol = rtol if adj_rtol is None else adj_rtol
        self.enable_adjoint(max(64, len(sensors)))
        options = (abi.ADJ_CHECKPOINT if checkpoint else 0) | (abi.ADJ_MIXED if mixed else 0)
        if mixed:
            self.enable_mixed()
        nbytes = C.c_size_t()
        _check(self.lib, self.h, self.lib.pt_adjoint_tape_size(self.h, int(n_steps), int(n_picard), options,
                                                               C.byref(nbytes)),
               "tape size")
        self.tape_bytes = nbytes.value
        with torch.cuda.stream(self.stream):
            tape = torch.empty((nbytes.value + 7) // 8, dtype=torch.float64, device=self.device)
        s_arr = np.ascontiguousarray(sensors, dtype=np.int64)
        d_arr = np.ascontiguousarray(d_obs, dtype=np.float64)
        J = C.c_double()
        fit = C.c_int64()
        ait = C.c_int64()
        st = _check(self.lib, self.h, self.lib.pt_adjoint_run(
            self.h, int(n_steps), int(n_picard), options, float(rtol), float(adj_rtol), int(max_iter),
            s_arr.ctypes.data_as(C.POINTER(C.c_int64)), len(s_arr), d_arr.ctypes.data_as(C.POINTER(C.c_double)),
            C.c_void_p(tape.data_ptr()), nbytes.value, C.c_void_p(self.grad_buf.data_ptr()),
            C.byref(J), C.byref(fit), C.byref(ait)), "adjoint_run")
        del tape
        if st != 0:
            raise abi.PTError(st, "adjoint_run: " + self.lib.pt_last_error(self.h).decode())
        return J.value, self.grad_buf[:self.nz, :self.ny, :self.nx], fit.value, ait.value

    def reset_state(self, phi):
        """Back to the initial state of every workload (pt_reset_state: V = R
        = 0, pressures and stress history 0, Mn = mu0, counters cleared),
        then ln(1-phi) from phi (pt_set_porosity), keeping k0."""
        _check(self.lib, self.h, self.lib.pt_reset_state(self.h), "reset_state")
        self.set_porosity(phi)

    def set_porosity(self, phi):
        """ln(1-phi) and its old value from a porosity array (nz, ny, nx) or
        device tensor (pt_set_porosity; PTError PT_EDOMAIN if phi leaves (0, 1))."""
        with torch.cuda.stream(self.stream):
            box = torch.zeros(self.buf["pt"][0].shape, dtype=torch.float64, device=self.device)
            box[:self.nz, :self.ny, :self.nx].copy_(torch.as_tensor(phi, dtype=torch.float64, device=self.device))
        _check(self.lib, self.h, self.lib.pt_set_porosity(self.h, C.c_void_p(box.data_ptr())), "set_porosity")

    def copy(self, src: torch.Tensor, dst: torch.Tensor):
        assert src.dtype == dst.dtype == torch.float64 and src.numel() == dst.numel()
        _check(self.lib, self.h, self.lib.pt_copy(self.h, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                                  src.numel()), "copy")

    def synchronize(self):
        self.stream.synchronize()
