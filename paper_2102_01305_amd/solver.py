"""Python binding of libibmlbm: argument marshalling only.

Every step of the time loop runs in the HIP kernels behind the C ABI; torch
supplies the device workspace (one uint8 tensor) and the HIP stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

_STORAGE = {"fp32": L.FP32, "fp16": L.FP16_DEV, "bf16": L.BF16_DEV}


def lattice_params(re, j, f, chord, kappa=0.2):
    """Clap & fling physics to lattice units through the library."""
    lib = L.load()
    out = [C.c_double() for _ in range(4)]
    L.check(lib.ibmlbm_lattice_params(re, j, f, chord, kappa, *[C.byref(o) for o in out]))
    tau, u_inf, u_tip, period = (o.value for o in out)
    return dict(tau=tau, u_inf=u_inf, u_tip=u_tip, period_steps=period)


def plate_params(re, u_inf, chord):
    """Fixed foil in a uniform stream to lattice units through the library."""
    lib = L.load()
    tau = C.c_double()
    L.check(lib.ibmlbm_plate_params(re, u_inf, chord, C.byref(tau)))
    return dict(tau=tau.value)


def figure_eight_params(re, u_tip, chord, a0):
    """Figure-eight stroke to lattice units through the library."""
    lib = L.load()
    tau, period = C.c_double(), C.c_double()
    L.check(lib.ibmlbm_figure_eight_params(re, u_tip, chord, a0, C.byref(tau), C.byref(period)))
    return dict(tau=tau.value, period_steps=period.value)


def complete_case(bx, wings, phys):
    """Fill tau, inlet velocity, reference velocity and periods of a workload
    description using the library's own parameter mapping."""
    bx = dict(bx)
    wings = [dict(w) for w in wings]
    if phys["kind"] == "plate":
        bx["tau"] = plate_params(phys["re"], phys["u_inf"], phys["chord"])["tau"]
        for w in wings:
            if w.get("period_steps") is None:
                w["period_steps"] = 1.0
    elif phys["kind"] == "clap_fling":
        p = lattice_params(phys["re"], phys["j"], phys["f"], phys["chord"], phys.get("kappa", 0.2))
        bx["tau"] = p["tau"]
        bx["u_in"] = [p["u_inf"], 0.0, 0.0]
        bx["u_ref"] = p["u_tip"]
        for w in wings:
            w["period_steps"] = p["period_steps"]
    elif phys["kind"] == "figure_eight":
        p = figure_eight_params(phys["re"], phys["u_tip"], phys["chord"], phys["a0"])
        bx["tau"] = p["tau"]
        bx["u_ref"] = phys["u_tip"]
        for w in wings:
            w["period_steps"] = p["period_steps"]
    else:
        raise ValueError(phys["kind"])
    return bx, wings


def make_config(bx, storage="fp32", check_interval=0, history_steps=1024):
    c = L.Config()
    c.nx, c.ny, c.nz = bx["nx"], bx["ny"], bx["nz"]
    for i, v in enumerate(bx["bc"]):
        c.bc[i] = int(v)
    c.tau = float(bx["tau"])
    for i, v in enumerate(bx.get("u_in") or (0.0, 0.0, 0.0)):
        c.u_in[i] = float(v)
    c.rho_out = float(bx.get("rho_out", 1.0))
    for i, v in enumerate(bx.get("body_force") or (0.0, 0.0, 0.0)):
        c.body_force[i] = float(v)
    c.storage = _STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.check_interval = int(check_interval)
    c.u_ref = float(bx.get("u_ref") or 1.0)
    c.area_ref = float(bx.get("area_ref") or 1.0)
    c.history_steps = int(history_steps)
    return c


def make_wings(wings):
    arr = (L.Wing * max(1, len(wings)))()
    for k, w in enumerate(wings):
        x = arr[k]
        x.chord, x.thickness, x.ds = w["chord"], w["thickness"], w.get("ds", 1.0)
        x.hinge[0], x.hinge[1] = w["hinge"]
        x.pivot_frac, x.theta0, x.sense = w["pivot_frac"], w["theta0"], w["sense"]
        x.alpha_shape = int(w["alpha_shape"])
        x.alpha_mean, x.alpha_amp = w.get("alpha_mean", 0.0), w.get("alpha_amp", 0.0)
        x.period_steps = w.get("period_steps") or 1.0
        x.phase = w.get("phase", 0.0)
        x.trans_amp, x.trans_angle = w.get("trans_amp", 0.0), w.get("trans_angle", 0.0)
    return arr


def _dptr(a):
    return a.ctypes.data_as(L._dp) if a is not None else None


class Solver:
    """One D3Q19 + IBM solve on one GPU (one handle, one workspace)."""

    def __init__(self, bx, wings=(), storage="fp32", check_interval=0, history_steps=1024,
                 device=None, stream=None, noalloc=False, nbytes=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("ibmlbm needs a ROCm GPU; torch.cuda.is_available() is False")
        self.lib = L.load()
        self.torch = torch
        self.device = torch.device(device or "cuda:0")
        self.bx = dict(bx)
        self.cfg = make_config(bx, storage, check_interval, history_steps)
        self.wings_desc = [dict(w) for w in wings]
        self._wings = make_wings(self.wings_desc)
        nw = len(self.wings_desc)
        # noalloc: the buffer holds the two lattice states only (the lattice
        # part of the workspace is an upper bound) and the library keeps every
        # other region in its static device scratch (ibmlbm_create_noalloc)
        # nbytes: a workspace size the caller already has from
        # workspace_bytes() for the same description (create checks it)
        if nbytes is None or noalloc:
            nbytes = self.lib.ibmlbm_workspace_bytes(C.byref(self.cfg), 0 if noalloc else nw, self._wings)
        if nbytes == 0:
            raise L.IbmlbmError(L.EINVAL, self.lib.ibmlbm_last_error(None).decode())
        self.nbytes = int(nbytes)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.h = L.Handle()
            create = self.lib.ibmlbm_create_noalloc if noalloc else self.lib.ibmlbm_create
            L.check(create(C.byref(self.cfg), C.c_void_p(self.ws.data_ptr()), self.nbytes,
                           C.c_void_p(self.stream.cuda_stream), C.byref(self.h)))
        if nw:
            L.check(self.lib.ibmlbm_set_kinematics(self.h, nw, self._wings), self.h)
        self.N = self.cfg.nx * self.cfg.ny * self.cfg.nz
        self.nw = nw

    # -- state ---------------------------------------------------------------
    def init_fields(self, rho=None, u=None, fdist=None, step0=0):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        f = None if fdist is None else np.ascontiguousarray(fdist, dtype=np.float64).reshape(-1)
        if r is not None and r.size != self.N:
            raise ValueError("rho must hold nx*ny*nz values")
        if v is not None and v.size != 3 * self.N:
            raise ValueError("u must hold 3*nx*ny*nz values")
        if f is not None and f.size != 19 * self.N:
            raise ValueError("fdist must hold 19*nx*ny*nz values")
        L.check(self.lib.ibmlbm_init_fields(self.h, _dptr(r), _dptr(v), _dptr(f), int(step0)), self.h)

    def set_stream(self, stream):
        """Enqueue this solve's work on `stream` from now on (a torch stream)."""
        L.check(self.lib.ibmlbm_set_stream(self.h, C.c_void_p(stream.cuda_stream)), self.h)
        self.stream = stream

    def step(self, n=1):
        L.check(self.lib.ibmlbm_step(self.h, int(n)), self.h)

    @property
    def step_count(self):
        return int(self.lib.ibmlbm_step_count(self.h))

    # -- outputs -------------------------------------------------------------
    def forces(self, first=0, count=None):
        if count is None:
            count = self.step_count - first
        out = np.empty((count, max(self.nw, 1), 8))
        L.check(self.lib.ibmlbm_forces(self.h, int(first), int(count), _dptr(out)), self.h)
        return out[:, : self.nw]

    def fields(self, which="u"):
        shape = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        key = {"rho": L.FIELD_RHO, "u": L.FIELD_U, "fdist": L.FIELD_FDIST}[which]
        n = {L.FIELD_RHO: 1, L.FIELD_U: 3, L.FIELD_FDIST: 19}[key]
        out = np.empty((n,) + shape)
        L.check(self.lib.ibmlbm_fields(self.h, key, _dptr(out)), self.h)
        return out[0] if key == L.FIELD_RHO else out

    def markers(self, which):
        key = {"X": L.MARKER_X, "U": L.MARKER_U, "B": L.MARKER_RHS, "duB": L.MARKER_DU,
               "rhoB": L.MARKER_RHO, "dA": L.MARKER_DA}[which]
        m = int(self.lib.ibmlbm_marker_count(self.h))
        out = np.empty((m, 3) if key in (L.MARKER_X, L.MARKER_U, L.MARKER_RHS, L.MARKER_DU) else (m,))
        L.check(self.lib.ibmlbm_markers(self.h, key, _dptr(out)), self.h)
        return out

    def mass(self):
        st = C.c_int64()
        m = C.c_double()
        L.check(self.lib.ibmlbm_mass(self.h, C.byref(st), C.byref(m)), self.h)
        return int(st.value), float(m.value)

    # -- timing --------------------------------------------------------------
    def enable_timing(self, every=1):
        """Bracket the kernels of one step in `every` with HIP events (0 = off)."""
        L.check(self.lib.ibmlbm_timing(self.h, int(every)), self.h)

    def read_timing(self):
        c = C.c_double()
        n = C.c_int64()
        cells = C.c_double()
        m = C.c_double()
        L.check(self.lib.ibmlbm_read_timing(self.h, C.byref(c), C.byref(n), C.byref(cells),
                                            C.byref(m)), self.h)
        return dict(collide_ms=c.value, collide_launches=int(n.value), collide_cells=cells.value,
                    marker_ms=m.value)

    @property
    def footprint(self):
        """Device bytes this solve holds (its workspace)."""
        return self.nbytes

    @property
    def bytes_per_cell(self):
        return int(self.lib.ibmlbm_bytes_per_cell(self.h))

    def close(self):
        if getattr(self, "h", None):
            L.check(self.lib.ibmlbm_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(bx, wings=(), storage="fp32", check_interval=0, history_steps=1024):
    """Device bytes a solve of this description needs (0 if it is invalid)."""
    lib = L.load()
    cfg = make_config(bx, storage, check_interval, history_steps)
    arr = make_wings(list(wings))
    return int(lib.ibmlbm_workspace_bytes(C.byref(cfg), len(wings), arr))


def step_batch(solvers, n=1):
    """Advance every solver by n steps in lock step, each stage of a step as
    one grouped launch over all of them (they must share one stream)."""
    solvers = list(solvers)
    if not solvers:
        return
    lib = solvers[0].lib
    arr = (L.Handle * len(solvers))(*[s.h for s in solvers])
    rc = lib.ibmlbm_step_batch(arr, len(solvers), int(n))
    if rc != L.OK:
        raise L.IbmlbmError(rc, lib.ibmlbm_last_error(None).decode())
