"""D3Q19 lattice Boltzmann BGK with Guo forcing, FP64 (oracle; test-only).

Arrays are laid out (q, z, y, x) for distributions and (d, z, y, x) for
vectors, component order d = (x, y, z).  Lattice units: dx = dt = 1.

The paper works on D2Q9 (Sec. 2.1, Eq. 5); the 3D version uses the textbook
D3Q19 set below with c_s^2 = 1/3 (Sec. 2.1 states c_s = c/sqrt(3)).
"""
from __future__ import annotations

import numpy as np

PERIODIC, WALL, VELOCITY, PRESSURE, ZH_VELOCITY, ZH_PRESSURE = 0, 1, 2, 3, 4, 5

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
        (Sec. 2.1: uniform-velocity inflow, atmospheric-pressure outflow);
      * ZH_VELOCITY / ZH_PRESSURE faces (x only): the Zou-He scheme of the
        paper's cylinder case (Sec. 3.1), applied by `zou_he` after the pull;
        boundary cells whose entering links touch a y or z wall keep the
        equilibrium ghost of VELOCITY / PRESSURE.
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
        if kind in (VELOCITY, ZH_VELOCITY):
            rg = rhoS[:, :, bxc]
            ug = np.broadcast_to(u_in[:, None, None], (3, nz, ny))
        elif kind in (PRESSURE, ZH_PRESSURE):
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
    for face in (0, 1):
        if bc[face] in (ZH_VELOCITY, ZH_PRESSURE):
            zou_he(f, bc, face, u_in, rho_out)
    return f


def zou_he(f, bc, face, u_in, rho_out):
    """Zou-He boundary cells of x face `face` (0: x = 0, 1: x = nx - 1), in
    place on the streamed f.  With n = +1 on the -x face and -1 on the +x
    face, the unknown populations are those with c_x = n.  Known sums:
    K = sum_{c_x=0} f + 2 sum_{c_x=-n} f.  Mass and normal momentum give
    rho (1 - n u_x) = K, so
      velocity face: u prescribed, rho = K / (1 - n u_x);
      pressure face: rho = rho_out, u_x = n (1 - K / rho), u_y = u_z = 0.
    Each unknown is its opposite plus the equilibrium difference,
      f_i = f_opp(i) + 2 w_i rho (c_i . u) / c_s^2 - c_iy N_y - c_iz N_z,
    where N_t = (1/2) sum_{c_x=0} c_t f - rho u_t / 3 fixes the transverse
    momentum to rho u_t.  Cells whose entering links touch a y or z wall are
    left as streamed (equilibrium ghost)."""
    _, nz, ny, nx = f.shape
    xb = 0 if face == 0 else nx - 1
    n = 1 if face == 0 else -1
    ys = slice(0, ny) if bc[2] == PERIODIC else slice(1, ny - 1)
    zs = slice(0, nz) if bc[4] == PERIODIC else slice(1, nz - 1)
    fb = f[:, zs, ys, xb]                     # (19, z, y) view of the boundary cells
    zero = C[:, 0] == 0
    K = fb[zero].sum(axis=0) + 2.0 * fb[C[:, 0] == -n].sum(axis=0)
    if bc[face] == ZH_VELOCITY:
        u = [float(u_in[0]), float(u_in[1]), float(u_in[2])]
        rho = K / (1.0 - n * u[0])
        ux, uy, uz = (np.full_like(K, v) for v in u)
    else:
        rho = np.full_like(K, float(rho_out))
        ux = n * (1.0 - K / rho)
        uy = np.zeros_like(K)
        uz = np.zeros_like(K)
    Ny = 0.5 * (C[zero, 1][:, None, None] * fb[zero]).sum(axis=0) - rho * uy / 3.0
    Nz = 0.5 * (C[zero, 2][:, None, None] * fb[zero]).sum(axis=0) - rho * uz / 3.0
    for i in np.nonzero(C[:, 0] == n)[0]:
        cu = C[i, 0] * ux + C[i, 1] * uy + C[i, 2] * uz
        fb[i] = fb[OPP[i]] + 2.0 * W[i] * rho * cu / CS2 - C[i, 1] * Ny - C[i, 2] * Nz
