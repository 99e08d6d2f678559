"""ctypes declarations of the C ABI in include/ptporo.h and include/ptwaves.h
(marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libptporo.so")

ABI_VERSION = 4

FIELDS = ("vx", "vy", "vz", "pt", "pf", "lp", "rx", "ry", "rz", "pto", "pfo", "lpo",
          "sxx", "syy", "szz", "sxy", "sxz", "syz", "fox", "foy", "foz", "mn", "k0",
          "kc", "eta", "mus")
FIELD_ID = {n: i for i, n in enumerate(FIELDS)}
NPING = 9

F_POWERLAW, F_DPCAP, F_K0FIELD, F_MECHOFF, F_FP32_TALL, F_DTS_RULE = 1, 2, 4, 8, 16, 32
ADJ_CHECKPOINT, ADJ_MIXED = 1, 2

STATUS = {0: "PT_OK", 1: "PT_ENOTCONV", -1: "PT_EINVAL", -2: "PT_EDEVICE",
          -3: "PT_EDIVERGED", -4: "PT_EDOMAIN", -5: "PT_ESTATE"}


class Params(C.Structure):
    _fields_ = [("version", C.c_int32), ("flags", C.c_uint32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("phi0", C.c_double), ("kmuf0", C.c_double),
                ("eta0", C.c_double), ("mu0", C.c_double), ("cmu", C.c_double),
                ("rhofg", C.c_double), ("rhosg", C.c_double),
                ("beta_phi", C.c_double), ("beta_d", C.c_double),
                ("alpha", C.c_double), ("B", C.c_double), ("G", C.c_double), ("R0", C.c_double),
                ("n_pow", C.c_double), ("tau0", C.c_double),
                ("coh", C.c_double), ("fric_deg", C.c_double), ("tau_y_min", C.c_double),
                ("dt", C.c_double), ("dtS", C.c_double), ("beta_n", C.c_double),
                ("rho_i", C.c_double), ("c_v", C.c_double), ("c_pf", C.c_double),
                ("damp_c", C.c_double), ("nup", C.c_int32), ("pad_", C.c_int32),
                ("r_eta", C.c_double), ("r_mu", C.c_double),
                ("shear_bg", C.c_double), ("xsi_w", C.c_double)]


class Norms(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("f", "rpt", "rpf", "dl", "dpt", "dpf", "dvz", "dv")]


class Counters(C.Structure):
    _fields_ = [("version", C.c_int32), ("refreshed", C.c_int32), ("iter", C.c_int64),
                ("ref_set", C.c_int32), ("mixed_copy", C.c_int32),
                ("ref_v", C.c_double), ("ref_p", C.c_double),
                ("cur", C.c_int32 * NPING), ("mixed_clean", C.c_int32),
                ("steps", C.c_int64), ("dt_cum", C.c_double), ("dts", C.c_double),
                ("r_stored", C.c_int32), ("v_prev", C.c_int32)]


EXPORTS = ["pt_create", "pt_destroy", "pt_field_elems", "pt_bind_field", "pt_workspace_size",
           "pt_bind_workspace", "pt_set_stream", "pt_set_progress", "pt_set_params", "pt_current", "pt_begin_step",
           "pt_refresh", "pt_iteration", "pt_iterate", "pt_last_norms", "pt_solve_linear", "pt_solve_linear_static",
           "pt_residual_reference", "pt_set_residual_reference",
           "pt_porosity_step", "pt_reset_state", "pt_set_porosity", "pt_get_counters", "pt_set_counters",
           "pt_picard_step", "pt_mixed_workspace_size", "pt_bind_mixed_workspace", "pt_residual",
           "pt_solve_mixed", "pt_adjoint_workspace_size", "pt_bind_adjoint_workspace", "pt_set_log_k0",
           "pt_misfit", "pt_adjoint_stage", "pt_adjoint_tape_size", "pt_adjoint_run", "pt_copy", "pt_status_str", "pt_last_error", "pt_abi_version",
           "pt_mg_workspace_size", "pt_bind_mg_workspace", "pt_mg_levels", "pt_solve_mg",
           "pt_sync_damped_residual"]

# Stage solvers of pt_picard_step and the multigrid hierarchy.
SOLVER_FP64, SOLVER_MIXED, SOLVER_MG = 0, 1, 2
MG_MAX_LEVELS = 12
MG_MAX_KRYLOV = 8


class MgParams(C.Structure):
    _fields_ = [("version", C.c_int32), ("levels", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("coarse_sweeps", C.c_int32), ("n_pt", C.c_int32), ("c_v", C.c_double), ("c_pf", C.c_double),
                ("krylov", C.c_int32), ("eta_mean", C.c_int32)]


def mg_params(levels=0, nu1=4, nu2=4, coarse_sweeps=50, n_pt=4, c_v=8.0, c_pf=6.1, krylov=0,
              eta_mean=2) -> MgParams:
    """Multigrid parameters (pt_mg_params).  Defaults, measured on the mixed
    workload at 511^3 (a Picard step of 5 stages to 1e-8): the smoother
    diverges at c_v = 5 and at n_pt = 2, so c_v = 8 keeps a margin (80
    V-cycles, 6.55 s, against 77 and 6.32 s at c_v = 6.1); n_pt = 6 would
    cost 5-25 % more cycles.  krylov = m > 0: Krylov acceleration of the
    cycles with m stored directions.  eta_mean: the geometric mean of eta_phi
    on coarse grids (the same cycle counts as the arithmetic one on the unit
    cube, 15 % fewer on the production box, and the porosity-wave run at
    127^3 lasts 13 converged steps instead of 7; harmonic means diverge)."""
    return MgParams(ABI_VERSION, int(levels), int(nu1), int(nu2), int(coarse_sweeps), int(n_pt),
                    float(c_v), float(c_pf), int(krylov), int(eta_mean))


# Reactive porosity waves (include/ptwaves.h).
WAVES_ABI_VERSION = 1
WAVES_FIELDS = ("xs", "pf", "phi", "dpfdt", "xs_old", "pf_old", "phi_old")
WAVES_FIELD_ID = {n: i for i, n in enumerate(WAVES_FIELDS)}
WAVES_NPING = 4


class WavesParams(C.Structure):
    _fields_ = [("version", C.c_int32), ("nup", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("phi0", C.c_double), ("k_muf0", C.c_double), ("eta", C.c_double),
                ("rho_f", C.c_double), ("rho_s", C.c_double), ("g", C.c_double),
                ("beta_d", C.c_double), ("beta_s", C.c_double), ("beta_f", C.c_double),
                ("tau", C.c_double), ("beta_x", C.c_double), ("delta_x", C.c_double), ("xs_max", C.c_double),
                ("dt", C.c_double), ("c_pf", C.c_double), ("phi_min", C.c_double), ("phi_max", C.c_double)]


WAVES_EXPORTS = ["pt_waves_create", "pt_waves_destroy", "pt_waves_field_elems", "pt_waves_bind_field",
                 "pt_waves_workspace_size", "pt_waves_bind_workspace", "pt_waves_set_stream", "pt_waves_current",
                 "pt_waves_begin_step", "pt_waves_iterate", "pt_waves_last_error", "pt_waves_solve_step",
                 "pt_waves_last_message"]

PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int64)
PROGRESS_PHASE = {0: "forward", 1: "reverse", 2: "recompute", 3: "stage"}

_lib = None


class PTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libptporo.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run __graft_entry__.build())")
    # torch first: the library must bind the HIP runtime torch loaded (torch
    # owns the memory and the streams); loaded first, it would map a second
    # runtime, and torch's own would then find no GPU
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P = C.POINTER
    vp = C.c_void_p
    lib.pt_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int64, P(Params), P(vp)]
    lib.pt_destroy.argtypes = [vp]
    lib.pt_field_elems.argtypes = [vp]
    lib.pt_field_elems.restype = C.c_int64
    lib.pt_bind_field.argtypes = [vp, C.c_int32, C.c_int32, vp]
    lib.pt_workspace_size.argtypes = [vp, P(C.c_size_t)]
    lib.pt_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    lib.pt_set_stream.argtypes = [vp, vp]
    lib.pt_set_progress.argtypes = [vp, PROGRESS_FN, vp]
    lib.pt_set_params.argtypes = [vp, P(Params)]
    lib.pt_current.argtypes = [vp, C.c_int32, P(C.c_int32)]
    lib.pt_begin_step.argtypes = [vp, C.c_int32]
    lib.pt_refresh.argtypes = [vp, C.c_double, C.c_double]
    lib.pt_iteration.argtypes = [vp, C.c_int32, C.c_int32]
    lib.pt_iterate.argtypes = [vp, C.c_int64]
    lib.pt_last_norms.argtypes = [vp, P(Norms)]
    lib.pt_solve_linear.argtypes = [vp, C.c_double, C.c_int64, P(C.c_int64), P(C.c_double)]
    lib.pt_solve_linear_static.argtypes = [vp, C.c_double, C.c_int64, P(C.c_int64), P(C.c_double)]
    lib.pt_porosity_step.argtypes = [vp]
    lib.pt_reset_state.argtypes = [vp]
    lib.pt_set_porosity.argtypes = [vp, vp]
    lib.pt_get_counters.argtypes = [vp, P(Counters)]
    lib.pt_set_counters.argtypes = [vp, P(Counters)]
    lib.pt_picard_step.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_int64, C.c_int32, C.c_double,
                                   P(C.c_int64), P(C.c_double)]
    lib.pt_residual_reference.argtypes = [vp, P(C.c_double), P(C.c_double)]
    lib.pt_set_residual_reference.argtypes = [vp, C.c_double, C.c_double]
    lib.pt_copy.argtypes = [vp, vp, vp, C.c_int64]
    lib.pt_mixed_workspace_size.argtypes = [vp, P(C.c_size_t)]
    lib.pt_bind_mixed_workspace.argtypes = [vp, vp, C.c_size_t]
    lib.pt_residual.argtypes = [vp]
    lib.pt_solve_mixed.argtypes = [vp, C.c_double, C.c_double, C.c_int64, C.c_int32,
                                   P(C.c_int64), P(C.c_int32), P(C.c_double)]
    lib.pt_adjoint_workspace_size.argtypes = [vp, C.c_int32, P(C.c_size_t)]
    lib.pt_bind_adjoint_workspace.argtypes = [vp, vp, C.c_size_t, C.c_int32]
    lib.pt_set_log_k0.argtypes = [vp, vp]
    lib.pt_misfit.argtypes = [vp, P(C.c_int64), C.c_int32, P(C.c_double), P(C.c_double)]
    lib.pt_adjoint_stage.argtypes = [vp, P(C.c_int64), C.c_int32, P(C.c_double), C.c_double, C.c_int64, vp,
                                     P(C.c_double), P(C.c_int64), P(C.c_double)]
    lib.pt_adjoint_tape_size.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, P(C.c_size_t)]
    lib.pt_adjoint_run.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int64,
                                   P(C.c_int64), C.c_int32, P(C.c_double), vp, C.c_size_t, vp,
                                   P(C.c_double), P(C.c_int64), P(C.c_int64)]
    lib.pt_sync_damped_residual.argtypes = [vp]
    lib.pt_mg_workspace_size.argtypes = [vp, P(MgParams), P(C.c_size_t)]
    lib.pt_bind_mg_workspace.argtypes = [vp, P(MgParams), vp, C.c_size_t]
    lib.pt_mg_levels.argtypes = [vp, P(C.c_int32), P(C.c_int32)]
    lib.pt_solve_mg.argtypes = [vp, C.c_double, C.c_int64, P(C.c_int64), P(C.c_double)]
    lib.pt_status_str.argtypes = [C.c_int]
    lib.pt_status_str.restype = C.c_char_p
    lib.pt_last_error.argtypes = [vp]
    lib.pt_last_error.restype = C.c_char_p
    lib.pt_abi_version.restype = C.c_int32
    for name in EXPORTS:
        if name not in ("pt_status_str", "pt_last_error", "pt_field_elems", "pt_abi_version"):
            getattr(lib, name).restype = C.c_int
    lib.pt_waves_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int64, P(WavesParams), P(vp)]
    lib.pt_waves_destroy.argtypes = [vp]
    lib.pt_waves_field_elems.argtypes = [vp]
    lib.pt_waves_field_elems.restype = C.c_int64
    lib.pt_waves_bind_field.argtypes = [vp, C.c_int32, C.c_int32, vp]
    lib.pt_waves_workspace_size.argtypes = [vp, P(C.c_size_t)]
    lib.pt_waves_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    lib.pt_waves_set_stream.argtypes = [vp, vp]
    lib.pt_waves_current.argtypes = [vp, C.c_int32, P(C.c_int32)]
    lib.pt_waves_begin_step.argtypes = [vp]
    lib.pt_waves_iterate.argtypes = [vp, C.c_int64]
    lib.pt_waves_last_error.argtypes = [vp, P(C.c_double)]
    lib.pt_waves_solve_step.argtypes = [vp, C.c_double, C.c_int64, P(C.c_int64), P(C.c_double)]
    lib.pt_waves_last_message.argtypes = [vp]
    lib.pt_waves_last_message.restype = C.c_char_p
    for name in WAVES_EXPORTS:
        if name not in ("pt_waves_field_elems", "pt_waves_last_message"):
            getattr(lib, name).restype = C.c_int
    if lib.pt_abi_version() != ABI_VERSION:
        raise ImportError("libptporo.so ABI version mismatch")
    _lib = lib
    return lib


def params_from(phys, k0field: bool) -> Params:
    """Marshal a Physics record into the C struct."""
    p = Params()
    p.version = ABI_VERSION
    flags = 0
    if phys.powerlaw:
        flags |= F_POWERLAW
    if phys.dpcap:
        flags |= F_DPCAP
    if k0field:
        flags |= F_K0FIELD
    if phys.mech_off:
        flags |= F_MECHOFF
    if getattr(phys, "fp32_tall", False):
        flags |= F_FP32_TALL
    if getattr(phys, "dts_rule", False):
        flags |= F_DTS_RULE
    p.flags = flags
    for name, ctype in Params._fields_:
        if ctype is C.c_double:
            setattr(p, name, float(getattr(phys, name)))
    p.nup = int(phys.nup)
    return p


def waves_params_from(phys) -> WavesParams:
    """Marshal a WavePhysics record into the C struct."""
    p = WavesParams()
    p.version = WAVES_ABI_VERSION
    p.nup = int(phys.nup)
    for name, ctype in WavesParams._fields_[2:]:
        setattr(p, name, float(getattr(phys, name)))
    return p
