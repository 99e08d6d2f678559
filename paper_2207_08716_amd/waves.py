"""Python handle over the reactive porosity-wave solver (include/ptwaves.h):
torch owns the device buffers and the stream, libptporo.so does every step of
the computation (thesis article 3; the appendix reactive script).

The fields live in one skewed allocation in the padded-box layout of the
two-phase solver, (k (ny+1) + j) pitch + i; only cells are used.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import abi

# Skew between consecutive field buffers (doubles), as for the two-phase grid.
FIELD_SKEW = 32


def _check(lib, h, st, what):
    if st < 0:
        msg = lib.pt_waves_last_message(h).decode() if h else ""
        raise abi.PTError(st, f"{what}: {msg}")
    return st


class Waves:
    """Reactive porosity-wave state on one GPU for an nx x ny x nz cell grid.

    phys: paper_2207_08716_amd.inputs.WavePhysics; phi: initial porosity
    (nz, ny, nx); Xs starts at xs_max/2 (or xs), Pf and dPf/dt at zero."""

    def __init__(self, phys, nx, ny, nz, phi, xs=None, device="cuda", stream=None):
        self.lib = abi.load()
        self.phys = phys
        self.nx, self.ny, self.nz = nx, ny, nz
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on the GPU only")
        self.pitch = ((nx + 1 + 31) // 32) * 32
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._params = abi.waves_params_from(phys)
        h = C.c_void_p()
        st = self.lib.pt_waves_create(nx, ny, nz, self.pitch, C.byref(self._params), C.byref(h))
        if st != 0:
            raise abi.PTError(st, "pt_waves_create rejected the grid or parameters")
        self.h = h
        _check(self.lib, h, self.lib.pt_waves_set_stream(h, C.c_void_p(self.stream.cuda_stream)), "set_stream")
        box = (nz + 1, ny + 1, self.pitch)
        nel = box[0] * box[1] * box[2]
        assert self.lib.pt_waves_field_elems(h) == nel
        count = abi.WAVES_NPING * 2 + len(abi.WAVES_FIELDS) - abi.WAVES_NPING
        stride = nel + FIELD_SKEW
        self.buf = {}
        with torch.cuda.stream(self.stream):
            self.arena = torch.zeros(count * stride + 32, dtype=torch.float64, device=self.device)
            base = (-self.arena.data_ptr() // 8) % 32
            k = 0
            for fid, name in enumerate(abi.WAVES_FIELDS):
                self.buf[name] = []
                for cp in range(2 if fid < abi.WAVES_NPING else 1):
                    off = base + k * stride
                    t = self.arena[off:off + nel].view(box)
                    self.buf[name].append(t)
                    _check(self.lib, h, self.lib.pt_waves_bind_field(h, fid, cp, C.c_void_p(t.data_ptr())),
                           f"bind {name}")
                    k += 1
            nbytes = C.c_size_t()
            _check(self.lib, h, self.lib.pt_waves_workspace_size(h, C.byref(nbytes)), "workspace_size")
            self.ws = torch.zeros((nbytes.value + 7) // 8, dtype=torch.float64, device=self.device)
            _check(self.lib, h, self.lib.pt_waves_bind_workspace(h, C.c_void_p(self.ws.data_ptr()), nbytes.value),
                   "bind workspace")
        self.set("phi", phi)
        self.set("xs", 0.5 * phys.xs_max if xs is None else xs)

    def close(self):
        if getattr(self, "h", None):
            self.lib.pt_waves_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state access --------------------------------------------------------
    def tensor(self, name):
        """Device tensor (padded box) holding the present value of a field."""
        cp = C.c_int32()
        _check(self.lib, self.h, self.lib.pt_waves_current(self.h, abi.WAVES_FIELD_ID[name], C.byref(cp)), "current")
        return self.buf[name][cp.value]

    def view(self, name):
        return self.tensor(name)[:self.nz, :self.ny, :self.nx]

    def get(self, name) -> np.ndarray:
        with torch.cuda.stream(self.stream):
            return self.view(name).cpu().numpy().copy()

    def set(self, name, value):
        with torch.cuda.stream(self.stream):
            v = self.view(name)
            if np.isscalar(value):
                v.fill_(float(value))
            else:
                a = np.ascontiguousarray(value, dtype=np.float64)
                assert a.shape == tuple(v.shape), (name, a.shape, tuple(v.shape))
                v.copy_(torch.from_numpy(a).to(self.device))

    # ---- the solver ------------------------------------------------------------
    def begin_step(self):
        _check(self.lib, self.h, self.lib.pt_waves_begin_step(self.h), "begin_step")

    def iterate(self, n):
        _check(self.lib, self.h, self.lib.pt_waves_iterate(self.h, int(n)), "iterate")

    def last_error(self) -> float:
        e = C.c_double()
        _check(self.lib, self.h, self.lib.pt_waves_last_error(self.h, C.byref(e)), "last_error")
        return e.value

    def solve_step(self, eps, iter_max):
        """Iterate until the stopping quantity is below eps (checked every
        nup iterations) or iter_max; returns (iterations, error, converged)."""
        it, e = C.c_int64(), C.c_double()
        st = self.lib.pt_waves_solve_step(self.h, float(eps), int(iter_max), C.byref(it), C.byref(e))
        _check(self.lib, self.h, st, "solve_step")
        return it.value, e.value, st == 0

    def synchronize(self):
        self.stream.synchronize()
