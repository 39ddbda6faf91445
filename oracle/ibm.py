"""Implicit velocity-correction immersed boundary method, FP64 (oracle; test-only).

Sec. 2.2 of the paper (after Wu & Shu): Lagrangian markers X_B^l carry an
unknown velocity correction du_B^l; it is spread to the lattice with the
4-point cosine delta kernel (Eqs. 12-15), and chosen so that the corrected
lattice velocity interpolated back to the markers equals the wall velocity
(Eqs. 16-19), i.e. the linear system A X = B is solved every time step.

3D readings (the paper is 2D):
  * D(x - X) = delta(x - X) delta(y - Y) delta(z - Z) (Eq. 13 with a third factor);
    the cell volume dx dy dz = 1 replaces dx dy in Eqs. 17-18.
  * the arc length ds_l of Eq. 15 becomes the surface element
    dA_l = (perimeter / n_perimeter) * dz with dz = 1 for a foil extruded over
    the periodic span, one marker layer per lattice plane at z = k + 1/2.
  * Eq. 18 repeats the index l in both kernels; the matrix entry is read as
    A_kl = dA_l sum_x D(x - X_k) D(x - X_l), k the row (constraint) marker.
  * With unit spanwise spacing the cosine kernel annihilates the alternating
    spanwise pattern (sum_j (-1)^j delta(j - X) = 0 for every X), so A is
    singular.  Every solution of A X = B spreads to the same lattice field
    (S n = 0 for n in the null space); the minimum-norm solution of
    (I I^T) y = B with du_B = y / dA is taken, which makes du_B unique.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.integrate import quad
from scipy.optimize import brentq

ALPHA_CONST, ALPHA_SIN, ALPHA_ABS_SIN = 0, 1, 2
PINV_RCOND = 1e-12       # singular values below this fraction of the largest are null modes
DENSE_MAX = 4096         # largest block solved by dense least squares


def delta(r):
    """Eq. 14: 4-point cosine kernel, (1 + cos(pi |r| / 2)) / 4 for |r| <= 2."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    return np.where(r <= 2.0, 0.25 * (1.0 + np.cos(0.5 * np.pi * r)), 0.0)


# ----------------------------------------------------------------- geometry --

def ellipse_arclength(a, b, phi):
    """Arc length of (a cos t, b sin t) from t = 0 to t = phi (quadrature)."""
    return quad(lambda t: math.hypot(a * math.sin(t), b * math.cos(t)), 0.0, phi,
                epsabs=1e-13, epsrel=1e-13, limit=200)[0]


def perimeter_markers(wing):
    """Markers on the elliptic section of one foil (Sec. 3.2-3.3: elliptic
    foil, aspect ratio = chord / thickness).

    Semi-axes a = chord/2 along the chord, b = thickness/2.  The leading edge
    is the local point (-a, 0), the trailing edge (+a, 0).  n = round(P / ds)
    markers at equal arc length, the first one at the trailing edge, going
    counter-clockwise in the local frame.  Returns (ref, ds_eff) where ref is
    (n, 2) coordinates relative to the pivot, which sits on the chord at
    fraction pivot_frac from the leading edge (0 = LE, 1/2 = centre, 1 = TE).
    """
    a = 0.5 * wing["chord"]
    b = 0.5 * wing["thickness"]
    P = ellipse_arclength(a, b, 2.0 * math.pi)
    n = max(3, int(round(P / wing["ds"])))
    step = P / n
    phis = [0.0]
    for j in range(1, n):
        target = j * step
        phis.append(brentq(lambda t: ellipse_arclength(a, b, t) - target,
                           0.0, 2.0 * math.pi, xtol=1e-14, rtol=1e-15))
    phis = np.array(phis)
    xp = -a + 2.0 * a * wing["pivot_frac"]
    ref = np.stack([a * np.cos(phis) - xp, b * np.sin(phis)], axis=1)
    return ref, step


def alpha(wing, t):
    """Angle-of-attack history and its time derivative.

    CONST: alpha_mean.  SIN: mean + amp sin(2 pi t/T + phase) (Eq. 21 with
    mean = pi/4, amp = -pi/4; Eq. 23 with mean = 0, amp = pi/3).
    ABS_SIN: mean + amp |sin(2 pi t/T + phase)|: the reading of Eq. 23 for
    clap & fling, whose text says alpha runs from 0 to 60 degrees.  At the
    kinks (|sin| = 0) the derivative is the one-sided value from later times.
    The kink position is found from the half-period phase
    h = psi - floor(2 psi)/2, psi = t/T + phase/(2 pi), so that every
    implementation taking the same floor lands on the same side.
    """
    shape = wing["alpha_shape"]
    mean, amp = wing["alpha_mean"], wing["alpha_amp"]
    if shape == ALPHA_CONST:
        return mean, 0.0
    T = wing["period_steps"]
    om = 2.0 * math.pi / T
    if shape == ALPHA_SIN:
        arg = om * t + wing["phase"]
        return mean + amp * math.sin(arg), amp * om * math.cos(arg)
    if shape == ALPHA_ABS_SIN:
        psi = t / T + wing["phase"] / (2.0 * math.pi)
        h = psi - math.floor(2.0 * psi) / 2.0
        return mean + amp * math.sin(2.0 * math.pi * h), amp * om * math.cos(2.0 * math.pi * h)
    raise ValueError("unknown alpha shape")


def hinge_motion(wing, t):
    """Pivot position and velocity.  Eq. 20: the pivot oscillates along the
    stroke plane at angle beta = trans_angle with A(t) = trans_amp cos(2 pi t/T + phase)."""
    hx, hy = wing["hinge"]
    A0 = wing["trans_amp"]
    if A0 == 0.0:
        return np.array([hx, hy]), np.zeros(2)
    T = wing["period_steps"]
    om = 2.0 * math.pi / T
    arg = om * t + wing["phase"]
    beta = wing["trans_angle"]
    e = np.array([math.cos(beta), math.sin(beta)])
    return np.array([hx, hy]) + A0 * math.cos(arg) * e, -A0 * om * math.sin(arg) * e


def marker_state(wing, ref, nz, t):
    """Positions X and wall velocities U_B of one foil's markers at time t.

    Chord angle theta(t) = theta0 + sense * alpha(t); X = X_h + R(theta) ref.
    U_B = dX_h/dt + theta_dot z x (X - X_h): the rotational velocity that the
    paper adds to the kinematic motion (Sec. 3.3).  Markers are ordered
    perimeter-major: index l = p * nz + k, z_k = k + 1/2.
    Returns X (m,3), U (m,3), hinge position (2,).
    """
    al, ald = alpha(wing, t)
    th = wing["theta0"] + wing["sense"] * al
    thd = wing["sense"] * ald
    Xh, Vh = hinge_motion(wing, t)
    c, s = math.cos(th), math.sin(th)
    rx = c * ref[:, 0] - s * ref[:, 1]
    ry = s * ref[:, 0] + c * ref[:, 1]
    n = ref.shape[0]
    X = np.empty((n, nz, 3))
    U = np.empty((n, nz, 3))
    X[:, :, 0] = (Xh[0] + rx)[:, None]
    X[:, :, 1] = (Xh[1] + ry)[:, None]
    X[:, :, 2] = (np.arange(nz) + 0.5)[None, :]
    U[:, :, 0] = (Vh[0] - thd * ry)[:, None]
    U[:, :, 1] = (Vh[1] + thd * rx)[:, None]
    U[:, :, 2] = 0.0
    return X.reshape(-1, 3), U.reshape(-1, 3), Xh


# ------------------------------------------------- interpolation / spreading --

def stencil(X, dims, periodic):
    """The 4 x 4 x 4 lattice nodes where D(x - X_l) can be non-zero.

    Per axis the nodes floor(X) - 1 .. floor(X) + 2 cover every node with
    |x - X| < 2 (Eq. 14 vanishes at |r| >= 2).  Periodic axes wrap; on other
    axes every node must lie inside the box.  Returns flat node indices
    (x fastest, then y, then z) and weights D = delta*delta*delta, both (m, 64).
    """
    X = np.asarray(X, dtype=np.float64)
    m = X.shape[0]
    nx, ny, nz = dims
    idx = []
    wts = []
    for d in range(3):
        base = np.floor(X[:, d]).astype(np.int64) - 1
        nodes = base[:, None] + np.arange(4)[None, :]
        w = delta(nodes - X[:, d][:, None])
        if periodic[d]:
            nodes = np.mod(nodes, dims[d])
        elif nodes.min() < 0 or nodes.max() >= dims[d]:
            raise ValueError("marker support leaves the box on a non-periodic axis")
        idx.append(nodes)
        wts.append(w)
    flat = (idx[2][:, :, None, None] * ny + idx[1][:, None, :, None]) * nx + idx[0][:, None, None, :]
    D = wts[2][:, :, None, None] * wts[1][:, None, :, None] * wts[0][:, None, None, :]
    return flat.reshape(m, 64), D.reshape(m, 64)


def interpolate(field_flat, nodes, weights):
    """Eq. 17 (first term): sum_x g(x) D(x - X_l) dV, dV = 1, as a gather.
    field_flat is (..., N); returns (..., m)."""
    return (field_flat[..., nodes] * weights).sum(axis=-1)


def spread(values, dA, nodes, weights, n_cells):
    """Eq. 15: g(x) = sum_l v_l D(x - X_l) dA_l, as a scatter-add.
    values is (d, m); returns (d, n_cells)."""
    values = np.atleast_2d(values)
    out = np.zeros((values.shape[0], n_cells))
    contrib = (values * dA[None, :])[:, :, None] * weights[None, :, :]
    for c in range(values.shape[0]):
        np.add.at(out[c], nodes.ravel(), contrib[c].ravel())
    return out


def interpolation_matrix(nodes, weights, n_cells):
    """The sparse operator I with I[l, x] = D(x - X_l) (m x N)."""
    m = nodes.shape[0]
    rows = np.repeat(np.arange(m), nodes.shape[1])
    return sp.csr_matrix((weights.ravel(), (rows, nodes.ravel())), shape=(m, n_cells))


def system_matrix(nodes, weights, dA, n_cells):
    """Eq. 18-19: A_kl = dA_l sum_x D(x - X_k) D(x - X_l) = (I I^T diag(dA))_kl.

    Returns (M, A) with M = I I^T (symmetric) and A = M diag(dA), sparse."""
    I = interpolation_matrix(nodes, weights, n_cells)
    M = (I @ I.T).tocsr()
    A = (M @ sp.diags(dA)).tocsr()
    return M, A


# ------------------------------------------------------------------- solve --

def _pinv_sym(Mb):
    return np.linalg.pinv(Mb, rcond=PINV_RCOND, hermitian=True)


def solve_dense(Mb, B):
    """Minimum-norm least-squares solution of Mb y = B by dense SVD, singular
    values below PINV_RCOND of the largest taken as zero."""
    return sla.lstsq(Mb.toarray() if sp.issparse(Mb) else Mb, B, cond=PINV_RCOND)[0]


def solve_block(Mb, B, tensor_shape=None, force_dense=False):
    """Minimum-norm solution y of Mb y = B (Mb symmetric PSD, B is (m, k)).

    Without a tensor shape (or with force_dense) the block is solved by dense
    least squares (solve_dense; at most DENSE_MAX markers).  An extruded foil
    has Mb = P (x) Q, P over its n_p perimeter markers and Q over its n_s span
    layers, because D is a product of 1D kernels; the structure is verified
    from the entries of Mb and the identity pinv(P (x) Q) = pinv(P) (x)
    pinv(Q) gives the same minimum-norm solution at a cost of n_p^3 + n_s^3.
    """
    m = Mb.shape[0]
    if tensor_shape is None or force_dense:
        if m > DENSE_MAX:
            raise ValueError("block too large for a dense solve and has no tensor structure")
        return solve_dense(Mb, B)
    n_p, n_s = tensor_shape
    Mb = sp.csr_matrix(Mb)
    q_ref = Mb[:n_s, :n_s].toarray()                   # = P[0,0] * Q
    p_ref = Mb[::n_s, ::n_s].toarray() / Mb[0, 0]       # = P / P[0,0]
    diff = sp.kron(sp.csr_matrix(p_ref), sp.csr_matrix(q_ref)) - Mb
    if diff.nnz and np.abs(diff.data).max() > 1e-13 * np.abs(Mb.data).max():
        raise ValueError("block is not a Kronecker product; no exact solve available")
    Pp = _pinv_sym(p_ref)
    Qp = _pinv_sym(q_ref)
    out = np.empty_like(B)
    for c in range(B.shape[1]):
        Y = Pp @ B[:, c].reshape(n_p, n_s) @ Qp.T
        out[:, c] = Y.ravel()
    return out


# ------------------------------------------------------------------ forces --

def wing_forces(rhoB, duB, dA, X, Xh, wing, u_ref, area_ref):
    """Eq. 26 and Sec. 3.6-3.7: Lagrangian force density f_B = 2 rho_B du_B / dt
    (dt = 1).  The force on the fluid is sum_l f_B dA_l; the force on the body
    is its negative.  Lift is the lateral (y) component, counted outward for a
    mirrored pair (sign -sense); thrust is -F_x (free stream along +x), drag
    = -thrust.  Coefficients divide by (1/2) rho_0 u_ref^2 area_ref (rho_0 = 1);
    the moment about the pivot divides additionally by the chord.
    Returns [Fx, Fy, Fz, Mz, CL, CT, CD, CM].
    """
    fb = -2.0 * rhoB[None, :] * duB * dA[None, :]      # (3, m) force on the body per marker
    F = fb.sum(axis=1)
    rx = X[:, 0] - Xh[0]
    ry = X[:, 1] - Xh[1]
    Mz = float((rx * fb[1] - ry * fb[0]).sum())
    qS = 0.5 * u_ref * u_ref * area_ref
    CL = -wing["sense"] * F[1] / qS
    CT = -F[0] / qS
    CD = F[0] / qS
    CM = Mz / (qS * wing["chord"])
    return np.array([F[0], F[1], F[2], Mz, CL, CT, CD, CM])
