"""The IB-LBM time loop, FP64 (oracle; test-only).

State: S, the post-collision distributions of the previous step (S^0 is the
equilibrium of the initial fields).  One step n, in the order of Sec. 2.2:

 1. stream S with the boundary rules -> pre-collision f (Eqs. 1, 7, left side)
 2. rho = sum f, u* = (sum c f + F_body / 2) / rho (Eqs. 2, 9, 11)
 3. marker positions and wall velocities at t = n (Eqs. 20-23)
 4. interpolate u* and rho to the markers; B = U_B - I u* (Eq. 19)
 5. solve A X = B for du_B (Eqs. 18-19; minimum-norm solution)
 6. spread du(x) = sum_l du_B D dA (Eq. 15); u = u* + du (Eq. 16);
    F = F_body + 2 rho du (Eq. 11 rearranged as in Eq. 26)
 7. collide with Guo forcing (Eqs. 4, 7, 8) -> S for the next step
 8. record the forces on every foil (Eq. 26, Sec. 3.7)

F_body is an optional uniform force density used by closed-form tests.
lattice="c" runs steps 1, 2 and 7 through clattice (the same operations in
plain C with OpenMP, for long runs on large boxes); the default is lattice.py.
"""
from __future__ import annotations

import numpy as np

from . import ibm


class Sim:
    def __init__(self, bx, wings=(), rho0=None, u0=None, lattice="numpy"):
        if lattice == "c":
            from . import clattice as lat
        elif lattice == "numpy":
            from . import lattice as lat
        else:
            raise ValueError("lattice must be 'numpy' or 'c'")
        self.lat = lat
        self.nx, self.ny, self.nz = bx["nx"], bx["ny"], bx["nz"]
        self.bc = list(bx["bc"])
        self.tau = float(bx["tau"])
        if not self.tau > 0.5:
            raise ValueError("tau must exceed 1/2")
        self.u_in = np.array(bx.get("u_in") or [0.0, 0.0, 0.0], dtype=np.float64)
        self.rho_out = float(bx.get("rho_out", 1.0))
        self.fbody = np.array(bx.get("body_force") or [0.0, 0.0, 0.0], dtype=np.float64)
        self.u_ref = float(bx.get("u_ref") or 1.0)
        self.area_ref = float(bx.get("area_ref") or 1.0)
        self.N = self.nx * self.ny * self.nz
        shape = (self.nz, self.ny, self.nx)
        rho = np.ones(shape) if rho0 is None else np.asarray(rho0, np.float64).reshape(shape)
        u = np.zeros((3,) + shape) if u0 is None else np.asarray(u0, np.float64).reshape((3,) + shape)
        self.S = self.lat.equilibrium(rho, u)
        self.n = 0
        per = self.lat.PERIODIC
        self.periodic = [self.bc[0] == per, self.bc[2] == per, self.bc[4] == per]
        self.wings = [dict(w) for w in wings]
        self.refs = []
        self.dA = []
        for w in self.wings:
            if not self.periodic[2]:
                raise ValueError("foils are extruded over a periodic span")
            ref, ds = ibm.perimeter_markers(w)
            self.refs.append(ref)
            self.dA.append(np.full(ref.shape[0] * self.nz, ds * 1.0))
        self.history = []
        self.last = {}

    # -- helpers -------------------------------------------------------------
    def markers(self, t):
        Xs, Us, hs = [], [], []
        for w, ref in zip(self.wings, self.refs):
            X, U, Xh = ibm.marker_state(w, ref, self.nz, t)
            Xs.append(X)
            Us.append(U)
            hs.append(Xh)
        return Xs, Us, hs

    def prestate(self):
        """Pre-collision f of the next step and its rho, u* (Eq. 2, 9, 11)."""
        f = self.lat.stream(self.S, self.bc, self.u_in, self.rho_out)
        rho, mom = self.lat.moments(f)
        ustar = (mom + 0.5 * self.fbody[:, None, None, None]) / rho
        return f, rho, ustar

    # -- one step ------------------------------------------------------------
    def step(self):
        f, rho, ustar = self.prestate()
        du = np.zeros_like(ustar)
        rec = []
        if self.wings:
            Xs, Us, hs = self.markers(float(self.n))
            X = np.concatenate(Xs)
            U = np.concatenate(Us)
            dA = np.concatenate(self.dA)
            nodes, wts = ibm.stencil(X, (self.nx, self.ny, self.nz), self.periodic)
            rho_f = rho.reshape(-1)
            us_f = ustar.reshape(3, -1)
            rhoB = ibm.interpolate(rho_f, nodes, wts)
            B = U - ibm.interpolate(us_f, nodes, wts).T            # (m, 3)
            M, _ = ibm.system_matrix(nodes, wts, dA, self.N)
            y = np.zeros_like(B)
            lo = 0
            for w, ref in zip(self.wings, self.refs):
                m_w = ref.shape[0] * self.nz
                hi = lo + m_w
                if M[lo:hi, :lo].nnz or M[lo:hi, hi:].nnz:
                    raise ValueError("marker supports of two foils overlap")
                y[lo:hi] = ibm.solve_block(M[lo:hi, lo:hi], B[lo:hi],
                                           tensor_shape=(ref.shape[0], self.nz))
                lo = hi
            duB = (y / dA[:, None]).T                               # (3, m)
            du = ibm.spread(duB, dA, nodes, wts, self.N).reshape(ustar.shape)
            lo = 0
            for k, (w, ref) in enumerate(zip(self.wings, self.refs)):
                hi = lo + ref.shape[0] * self.nz
                rec.append(ibm.wing_forces(rhoB[lo:hi], duB[:, lo:hi], dA[lo:hi],
                                           X[lo:hi], hs[k], w, self.u_ref, self.area_ref))
                lo = hi
            self.last = dict(X=X, U=U, B=B, rhoB=rhoB, duB=duB, du=du, nodes=nodes,
                             wts=wts, dA=dA, rho=rho, ustar=ustar)
        u = ustar + du
        F = self.fbody[:, None, None, None] + 2.0 * rho[None] * du
        self.S = self.lat.collide(f, rho, u, F, self.tau)
        self.history.append(np.array(rec) if rec else np.zeros((0, 8)))
        self.n += 1

    def run(self, n):
        for _ in range(n):
            self.step()

    # -- outputs ---------------------------------------------------------------
    def fields(self):
        """rho and u* of the current state (what the next step starts from)."""
        _, rho, ustar = self.prestate()
        return rho, ustar

    def forces(self):
        """History [step][wing][8] (Fx, Fy, Fz, Mz, CL, CT, CD, CM)."""
        return np.array(self.history)

    def mass(self):
        return float(self.S.sum())
