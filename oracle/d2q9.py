"""The paper's own 2D scheme, FP64 (oracle; test-only): D2Q9 BGK with Guo
forcing (Sec. 2.1, Eqs. 1-9 with the Eq. 5 weights) coupled to the implicit
IBM on the perimeter markers of 2D elliptic foils (Sec. 2.2, Eqs. 13-19,
26), written independently of the D3Q19 oracle so that it can pin the
reduction of D3Q19 on one periodic layer to D2Q9.

Arrays are (q, y, x) for distributions and (d, y, x) for vectors, d = (x, y).
Boundary kinds per face (-x, +x, -y, +y) as in the 3D oracle: PERIODIC,
WALL (half-way bounce-back), VELOCITY / PRESSURE (equilibrium ghost from the
boundary cell), ZH_VELOCITY / ZH_PRESSURE (Zou-He; cells whose entering
links touch a wall keep the equilibrium ghost).
"""
from __future__ import annotations

import math

import numpy as np

from . import ibm
from .lattice import PERIODIC, PRESSURE, VELOCITY, WALL, ZH_PRESSURE, ZH_VELOCITY

# Eq. 5: rest, four axis neighbours, four diagonals
C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
             dtype=np.int64)
W = np.array([4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4)
Q = 9
OPP = np.array([int(np.nonzero((C == -C[i]).all(axis=1))[0][0]) for i in range(Q)])


def equilibrium(rho, u):
    """Second-order equilibrium, c_s^2 = 1/3 (Eq. 4 read as the standard form)."""
    cu = np.einsum("qd,d...->q...", C.astype(np.float64), u)
    usq = (u * u).sum(axis=0)
    return W.reshape((Q,) + (1,) * rho.ndim) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)


def guo(u, F, tau):
    """Eq. 8 with the c_i factor: (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F."""
    cu = np.einsum("qd,d...->q...", C.astype(np.float64), u)
    cF = np.einsum("qd,d...->q...", C.astype(np.float64), F)
    uF = (u * F).sum(axis=0)
    return (1.0 - 0.5 / tau) * W.reshape((Q,) + (1,) * uF.ndim) * (3.0 * (cF - uF) + 9.0 * cu * cF)


def moments(f):
    return f.sum(axis=0), np.einsum("qd,q...->d...", C.astype(np.float64), f)


def stream(S, bc, u_in, rho_out):
    """f_i(x) = S_i(x - c_i) with the boundary rules of the module docstring."""
    _, ny, nx = S.shape
    rhoS, momS = moments(S)
    u_in = np.asarray(u_in, dtype=np.float64)[:2]
    ghost = {}
    for face, xb in ((0, 0), (1, nx - 1)):
        if bc[face] in (VELOCITY, ZH_VELOCITY):
            ghost[face] = equilibrium(rhoS[:, xb], np.broadcast_to(u_in[:, None], (2, ny)))
        elif bc[face] in (PRESSURE, ZH_PRESSURE):
            ghost[face] = equilibrium(np.full(ny, float(rho_out)), momS[:, :, xb] / rhoS[None, :, xb])
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    f = np.empty_like(S)
    for i in range(Q):
        sx, sy = xx - C[i, 0], yy - C[i, 1]
        if bc[0] == PERIODIC:
            sx = np.mod(sx, nx)
        if bc[2] == PERIODIC:
            sy = np.mod(sy, ny)
        wall = np.zeros_like(xx, dtype=bool)
        if bc[0] == WALL:
            wall |= sx < 0
        if bc[1] == WALL:
            wall |= sx >= nx
        if bc[2] == WALL:
            wall |= sy < 0
        if bc[3] == WALL:
            wall |= sy >= ny
        cx, cy = np.clip(sx, 0, nx - 1), np.clip(sy, 0, ny - 1)
        val = S[i][cy, cx]
        if 0 in ghost:
            val = np.where(sx < 0, ghost[0][i][cy], val)
        if 1 in ghost:
            val = np.where(sx >= nx, ghost[1][i][cy], val)
        f[i] = np.where(wall, S[OPP[i]], val)
    for face in (0, 1):
        if bc[face] in (ZH_VELOCITY, ZH_PRESSURE):
            _zou_he(f, bc, face, u_in, rho_out)
    return f


def _zou_he(f, bc, face, u_in, rho_out):
    """Zou-He on the boundary column: with n the c_x of the entering
    populations, K = sum_{c_x=0} f + 2 sum_{c_x=-n} f and rho (1 - n u_x) = K;
    each unknown f_i = f_opp(i) + 6 w_i rho (c_i.u) - c_iy N_y, with
    N_y = (1/2) sum_{c_x=0} c_y f - rho u_y / 3."""
    _, ny, nx = f.shape
    xb, n = (0, 1) if face == 0 else (nx - 1, -1)
    ys = slice(0, ny) if bc[2] == PERIODIC else slice(1, ny - 1)
    fb = f[:, ys, xb]
    zero = C[:, 0] == 0
    K = fb[zero].sum(axis=0) + 2.0 * fb[C[:, 0] == -n].sum(axis=0)
    if bc[face] == ZH_VELOCITY:
        ux, uy = np.full_like(K, u_in[0]), np.full_like(K, u_in[1])
        rho = K / (1.0 - n * ux)
    else:
        rho = np.full_like(K, float(rho_out))
        ux, uy = n * (1.0 - K / rho), np.zeros_like(K)
    Ny = 0.5 * (C[zero, 1][:, None] * fb[zero]).sum(axis=0) - rho * uy / 3.0
    for i in np.nonzero(C[:, 0] == n)[0]:
        fb[i] = fb[OPP[i]] + 6.0 * W[i] * rho * (C[i, 0] * ux + C[i, 1] * uy) - C[i, 1] * Ny


# ------------------------------------------------------------------- IBM --

def _stencil2(X, nx, ny, periodic):
    """4 x 4 support nodes and weights delta(x - X) delta(y - Y) (Eqs. 13-14)."""
    m = X.shape[0]
    idx, wts = [], []
    for d, n in ((0, nx), (1, ny)):
        base = np.floor(X[:, d]).astype(np.int64) - 1
        nodes = base[:, None] + np.arange(4)[None, :]
        w = ibm.delta(nodes - X[:, d][:, None])
        if periodic[d]:
            nodes = np.mod(nodes, n)
        idx.append(nodes)
        wts.append(w)
    flat = idx[1][:, :, None] * nx + idx[0][:, None, :]
    D = wts[1][:, :, None] * wts[0][:, None, :]
    return flat.reshape(m, 16), D.reshape(m, 16)


class Sim2D:
    """The 2D method step by step (same order as the 3D oracle's Sim):
    stream, moments, markers at t = n, interpolate, B = U_B - I u*, solve
    (I I^T) y = B (dense; the 2D perimeter block is nonsingular), du_B =
    y / dA, spread, u = u* + du, F = F_body + 2 rho du, collide, forces."""

    def __init__(self, bx, wings=(), rho0=None, u0=None):
        self.nx, self.ny = bx["nx"], bx["ny"]
        self.bc = [bx["bc"][k] for k in range(4)]
        self.tau = float(bx["tau"])
        self.u_in = np.array((bx.get("u_in") or [0.0, 0.0, 0.0])[:2], dtype=np.float64)
        self.rho_out = float(bx.get("rho_out", 1.0))
        self.fbody = np.array((bx.get("body_force") or [0.0, 0.0, 0.0])[:2], dtype=np.float64)
        self.u_ref = float(bx.get("u_ref") or 1.0)
        self.area_ref = float(bx.get("area_ref") or 1.0)
        shape = (self.ny, self.nx)
        rho = np.ones(shape) if rho0 is None else np.asarray(rho0, np.float64).reshape(shape)
        u = np.zeros((2,) + shape) if u0 is None else np.asarray(u0, np.float64).reshape((2,) + shape)
        self.S = equilibrium(rho, u)
        self.n = 0
        self.wings = [dict(w) for w in wings]
        self.refs, self.ds = [], []
        for w in self.wings:
            ref, ds = ibm.perimeter_markers(w)
            self.refs.append(ref)
            self.ds.append(ds)
        self.history = []

    def _prestate(self):
        f = stream(self.S, self.bc, self.u_in, self.rho_out)
        rho, mom = moments(f)
        return f, rho, (mom + 0.5 * self.fbody[:, None, None]) / rho

    def step(self):
        f, rho, ustar = self._prestate()
        N = self.nx * self.ny
        per = (self.bc[0] == PERIODIC, self.bc[2] == PERIODIC)
        du = np.zeros_like(ustar)
        rows = []
        for w, ref, ds in zip(self.wings, self.refs, self.ds):
            X3, U3, Xh = ibm.marker_state(w, ref, 1, float(self.n))
            X, U = X3[:, :2], U3[:, :2]
            nodes, D = _stencil2(X, self.nx, self.ny, per)
            rhoB = (rho.reshape(N)[nodes] * D).sum(axis=1)
            ut = np.stack([(ustar[d].reshape(N)[nodes] * D).sum(axis=1) for d in range(2)], axis=1)
            B = U - ut
            Imat = np.zeros((X.shape[0], N))
            np.add.at(Imat, (np.repeat(np.arange(X.shape[0]), 16), nodes.ravel()), D.ravel())
            M = Imat @ Imat.T
            y = np.linalg.solve(M, B)
            duB = y / ds
            for d in range(2):
                np.add.at(du[d].reshape(N), nodes.ravel(), (D * (duB[:, d] * ds)[:, None]).ravel())
            fB = 2.0 * rhoB[:, None] * duB
            Fb = -(fB * ds).sum(axis=0)
            r = X - Xh[None, :]
            Mz = -((r[:, 0] * fB[:, 1] - r[:, 1] * fB[:, 0]) * ds).sum()
            qS = 0.5 * self.u_ref ** 2 * self.area_ref
            rows.append([Fb[0], Fb[1], 0.0, Mz, -w["sense"] * Fb[1] / qS, -Fb[0] / qS,
                         Fb[0] / qS, Mz / (qS * w["chord"])])
        u = ustar + du
        F = self.fbody[:, None, None] + 2.0 * rho[None] * du
        self.S = f - (f - equilibrium(rho, u)) / self.tau + guo(u, F, self.tau)
        self.history.append(rows)
        self.n += 1

    def run(self, n):
        for _ in range(n):
            self.step()

    def fields(self):
        """rho and u* of the state the next step starts from."""
        _, rho, ustar = self._prestate()
        return rho, ustar

    def forces(self):
        return np.array(self.history)
