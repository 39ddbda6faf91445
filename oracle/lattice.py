"""D3Q19 lattice Boltzmann BGK with Guo forcing, FP64 (oracle; test-only).

Arrays are laid out (q, z, y, x) for distributions and (d, z, y, x) for
vectors, component order d = (x, y, z).  Lattice units: dx = dt = 1.

The paper works on D2Q9 (Sec. 2.1, Eq. 5); the 3D version uses the textbook
D3Q19 set below with c_s^2 = 1/3 (Sec. 2.1 states c_s = c/sqrt(3)).
"""
from __future__ import annotations

import numpy as np

PERIODIC, WALL, VELOCITY, PRESSURE = 0, 1, 2, 3

# D3Q19 velocities: rest, 6 face neighbours, 12 edge neighbours.
C = np.array([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1],
], dtype=np.int64)
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
CS2 = 1.0 / 3.0
Q = 19
# opposite direction: C[OPP[i]] == -C[i]
OPP = np.array([int(np.nonzero((C == -C[i]).all(axis=1))[0][0]) for i in range(Q)])


def _bw(a, nd):
    """Reshape a length-19 table so it broadcasts against (19, ...) fields."""
    return a.reshape((Q,) + (1,) * nd)


def moments(f):
    """Eq. 2: rho = sum_i f_i and the momentum sum_i c_i f_i."""
    rho = f.sum(axis=0)
    mom = np.einsum("qd,q...->d...", C.astype(np.float64), f)
    return rho, mom


def equilibrium(rho, u):
    """Eq. 4, read as the standard second-order expansion of the Maxwellian:
    f_i^eq = w_i rho [1 + c_i.u/cs^2 + (c_i.u)^2/(2 cs^4) - u.u/(2 cs^2)].
    (The printed equation has (c_i - u)^2 and a bare u; those terms cannot be
    dimensionally right, and this is the form of the cited LBM literature.)
    """
    nd = rho.ndim
    cu = np.einsum("qd,d...->q...", C.astype(np.float64), u)
    usq = (u * u).sum(axis=0)
    return _bw(W, nd) * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2)
                               - usq / (2.0 * CS2))


def guo_source(u, F, tau):
    """Eq. 8 with the c_i factor on the second term restored (Guo et al.):
    F_i = (1 - 1/(2 tau)) w_i [(c_i - u)/cs^2 + (c_i.u) c_i / cs^4] . F,
    evaluated with the force-corrected velocity u of Eqs. 9-10.
    """
    nd = u.ndim - 1
    Cf = C.astype(np.float64)
    cu = np.einsum("qd,d...->q...", Cf, u)
    cF = np.einsum("qd,d...->q...", Cf, F)
    uF = (u * F).sum(axis=0)
    return (1.0 - 0.5 / tau) * _bw(W, nd) * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2))


def collide(f, rho, u, F, tau):
    """Eq. 7: post-collision f* = f - (f - f^eq)/tau + F_i (dt = 1)."""
    return f - (f - equilibrium(rho, u)) / tau + guo_source(u, F, tau)


def stream(S, bc, u_in, rho_out):
    """Streaming (left-hand side of Eqs. 1 and 7) with the boundary rules.

    S is the post-collision state (19, nz, ny, nx).  Returns the pre-collision
    state f with f_i(x) = S_i(x - c_i) where the source lies in the box.
    When the source x - c_i lies outside:
      * periodic axes wrap;
      * across a WALL face (any axis): half-way bounce-back of a resting wall,
        f_i(x) = S_opp(i)(x) (Sec. 2.1: walls by bounce-back).  A link that
        leaves through a wall and an inlet/outlet face at once takes this rule;
      * across a VELOCITY face (x only): equilibrium of the prescribed
        velocity u_in and of the density of S at the adjacent boundary cell;
      * across a PRESSURE face (x only): equilibrium of density rho_out and of
        the velocity of S at the adjacent boundary cell
        (Sec. 2.1: uniform-velocity inflow, atmospheric-pressure outflow).
    bc lists the six faces (-x, +x, -y, +y, -z, +z).
    """
    q, nz, ny, nx = S.shape
    dims = (nx, ny, nz)
    per = [bc[0] == PERIODIC, bc[2] == PERIODIC, bc[4] == PERIODIC]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cell = (xx, yy, zz)
    rhoS, momS = moments(S)
    u_in = np.asarray(u_in, dtype=np.float64)
    # equilibrium ghost layers at x = -1 and x = nx, one value per (z, y):
    # the missing moment comes from the boundary cell (x = 0 or nx - 1) of S
    ghost = {}
    for face, bxc in ((0, 0), (1, nx - 1)):
        kind = bc[face]
        if kind == VELOCITY:
            rg = rhoS[:, :, bxc]
            ug = np.broadcast_to(u_in[:, None, None], (3, nz, ny))
        elif kind == PRESSURE:
            rg = np.full((nz, ny), float(rho_out))
            ug = momS[:, :, :, bxc] / rhoS[None, :, :, bxc]
        else:
            continue
        ghost[face] = equilibrium(rg, ug)
    f = np.empty_like(S)
    for i in range(Q):
        src = []
        out_lo = []
        out_hi = []
        for d in range(3):
            s = cell[d] - C[i, d]
            if per[d]:
                s = np.mod(s, dims[d])
            out_lo.append(s < 0)
            out_hi.append(s >= dims[d])
            src.append(np.clip(s, 0, dims[d] - 1))
        wall = np.zeros(xx.shape, dtype=bool)
        for d in range(3):
            if bc[2 * d] == WALL:
                wall |= out_lo[d]
            if bc[2 * d + 1] == WALL:
                wall |= out_hi[d]
        sx, sy, sz = src
        val = S[i][sz, sy, sx]
        for face, mask in ((0, out_lo[0]), (1, out_hi[0])):
            if face in ghost:
                val = np.where(mask, ghost[face][i][sz, sy], val)
        f[i] = np.where(wall, S[OPP[i]], val)
    return f
