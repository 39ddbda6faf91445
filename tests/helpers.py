"""Shared set-up for tests: builds the same seeded workload for the oracle and
for the GPU solver.  Each side maps physics to lattice units itself."""
from __future__ import annotations

import numpy as np

import workloads as WL


def plate(nz=32, seed=0, **kw):
    """The small parity workload: 64x32x32 channel, fixed elliptic plate (c=10,
    aspect 5, 30 deg), inlet u=0.02, Re=100, noise 1e-4."""
    bx, wg, ph = WL.plate_case(nz=nz, **kw)
    shape = (bx["nz"], bx["ny"], bx["nx"])
    u0 = WL.velocity_noise(shape, seed)
    u0[0] += ph["u_inf"]
    return bx, wg, ph, u0


def clap_fling(seed=0, **kw):
    bx, wg, ph = WL.clap_fling_case(**kw)
    shape = (bx["nz"], bx["ny"], bx["nx"])
    u0 = WL.velocity_noise(shape, seed)
    return bx, wg, ph, u0


def oracle_sim(bx, wg, ph, u0=None, rho0=None, step0=0):
    from oracle import params
    from oracle.sim import Sim

    if ph is not None:
        bx, wg = params.complete_case(bx, wg, ph)
    u = None if u0 is None else u0.copy()
    if ph is not None and ph["kind"] == "clap_fling" and u is not None:
        u[0] += bx["u_in"][0]
    s = Sim(bx, wg, rho0=rho0, u0=u)
    s.n = step0
    return s


def gpu_solver(bx, wg, ph, u0=None, rho0=None, step0=0, storage="fp32", check_interval=0,
               history_steps=4096):
    from paper_2102_01305_amd.solver import Solver, complete_case

    if ph is not None:
        bx, wg = complete_case(bx, wg, ph)
    u = None if u0 is None else u0.copy()
    if ph is not None and ph["kind"] == "clap_fling" and u is not None:
        u[0] += bx["u_in"][0]
    s = Solver(bx, wg, storage=storage, check_interval=check_interval, history_steps=history_steps)
    s.init_fields(rho=rho0, u=u, step0=step0)
    return s


def l2rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# Force-history columns: Fx, Fy, Fz, Mz (moment about the pivot), CL, CT, CD, CM.
COEFFS = {"mz": 3, "cl": 4, "ct": 5, "cd": 6, "cm": 7}


def coeff_errors(fg, fo, names=("mz", "cl", "ct", "cd", "cm")):
    """Per history column: max over foils and steps of |gpu - ref| / max|ref|
    (the per-step rule, normalised by the largest reference value so zero
    crossings are not amplified)."""
    out = {}
    for k in names:
        c = COEFFS[k]
        out[k] = max(float(np.abs(fg[:, w, c] - fo[:, w, c]).max() / np.abs(fo[:, w, c]).max())
                     for w in range(fo.shape[1]))
    return out


def node_box_error(u_g, u_o, nodes):
    """Element-wise error of u on the cells the markers' kernel supports
    cover (flat cell indices `nodes`, e.g. the oracle's last stencil): max
    over those cells and components of |gpu - ref|, relative to max |ref|
    there.  About 3% of the cells of a clap & fling box lie there, so an
    error confined to them is diluted in a global L2 norm."""
    idx = np.unique(np.asarray(nodes).ravel())
    a = u_g.reshape(3, -1)[:, idx]
    b = u_o.reshape(3, -1)[:, idx]
    return float(np.abs(a - b).max() / np.abs(b).max())
