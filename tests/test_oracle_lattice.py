"""Pins of the oracle's lattice part against facts fixed by the mathematics.

Every check here is independent of the oracle's own formulas: lattice-tensor
identities, moment identities, exact invariants of the discrete dynamics and
closed-form flows (Poiseuille, Taylor-Green decay).
"""
import math

import numpy as np
import pytest

from oracle import lattice as L
from oracle.sim import Sim

P, Wl, V, PR = L.PERIODIC, L.WALL, L.VELOCITY, L.PRESSURE


def _box(nx, ny, nz, bc, tau, **kw):
    d = dict(nx=nx, ny=ny, nz=nz, bc=bc, tau=tau, u_in=[0, 0, 0], rho_out=1.0,
             body_force=[0, 0, 0], u_ref=1.0, area_ref=1.0)
    d.update(kw)
    return d


def test_d3q19_tensor_identities():
    C = L.C.astype(float)
    w = L.W
    assert L.Q == 19 and C.shape == (19, 3)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("q,qa->a", w, C), 0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("q,qa,qb->ab", w, C, C), np.eye(3) / 3, atol=1e-15)
    np.testing.assert_allclose(np.einsum("q,qa,qb,qc->abc", w, C, C, C), 0, atol=1e-15)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    np.testing.assert_allclose(np.einsum("q,qa,qb,qc,qd->abcd", w, C, C, C, C), iso, atol=1e-15)
    for i in range(19):
        assert (C[L.OPP[i]] == -C[i]).all()
    # speeds: 1 rest, 6 of length 1, 12 of length sqrt 2
    n2 = (C * C).sum(1)
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [2] * 12


def test_equilibrium_moments():
    rng = np.random.default_rng(1)
    rho = 1 + 0.1 * rng.standard_normal(50)
    u = 0.1 * rng.standard_normal((3, 50))
    feq = L.equilibrium(rho, u)
    C = L.C.astype(float)
    np.testing.assert_allclose(feq.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("qa,qn->an", C, feq), rho * u, atol=1e-15)
    Pi = np.einsum("qa,qb,qn->abn", C, C, feq)
    ref = rho[None, None] * (np.eye(3)[:, :, None] / 3 + u[:, None] * u[None, :])
    np.testing.assert_allclose(Pi, ref, atol=1e-15)


def test_guo_source_moments():
    rng = np.random.default_rng(2)
    u = 0.1 * rng.standard_normal((3, 40))
    F = 1e-3 * rng.standard_normal((3, 40))
    tau = 0.73
    Fi = L.guo_source(u, F, tau)
    C = L.C.astype(float)
    k = 1 - 0.5 / tau
    np.testing.assert_allclose(Fi.sum(0), 0, atol=1e-18)
    np.testing.assert_allclose(np.einsum("qa,qn->an", C, Fi), k * F, atol=1e-17)
    second = np.einsum("qa,qb,qn->abn", C, C, Fi)
    ref = k * (u[:, None] * F[None, :] + F[:, None] * u[None, :])
    np.testing.assert_allclose(second, ref, atol=1e-17)


def test_uniform_equilibrium_is_fixed_point_periodic():
    u0 = np.zeros((3, 5, 6, 7))
    u0[0], u0[1], u0[2] = 0.03, -0.02, 0.01
    s = Sim(_box(7, 6, 5, [P] * 6, 0.8), rho0=np.full((5, 6, 7), 1.02), u0=u0)
    S0 = s.S.copy()
    s.run(3)
    np.testing.assert_allclose(s.S, S0, rtol=0, atol=1e-15)


def test_uniform_flow_is_fixed_point_with_inlet_outlet():
    U = 0.04
    u0 = np.zeros((3, 4, 6, 9))
    u0[0] = U
    s = Sim(_box(9, 6, 4, [V, PR, P, P, P, P], 0.7, u_in=[U, 0, 0]), u0=u0)
    S0 = s.S.copy()
    s.run(4)
    np.testing.assert_allclose(s.S, S0, rtol=0, atol=1e-15)


def test_channel_wall_rest_state_with_inlet_outlet_at_rest():
    # fluid at rest, inlet velocity 0, walls in y: nothing moves
    s = Sim(_box(8, 5, 3, [V, PR, Wl, Wl, P, P], 0.9))
    S0 = s.S.copy()
    s.run(3)
    np.testing.assert_allclose(s.S, S0, atol=1e-16)


@pytest.mark.parametrize("bc", [[P] * 6, [Wl, Wl, Wl, Wl, P, P], [Wl] * 6, [P, P, Wl, Wl, Wl, Wl]])
def test_mass_conservation_closed_box(bc):
    rng = np.random.default_rng(3)
    shape = (6, 7, 8)
    rho0 = 1 + 0.01 * rng.standard_normal(shape)
    u0 = 0.02 * rng.standard_normal((3,) + shape)
    s = Sim(_box(8, 7, 6, bc, 0.62), rho0=rho0, u0=u0)
    m0 = s.mass()
    s.run(60)
    assert abs(s.mass() - m0) <= 1e-13 * m0
    assert abs(m0 - rho0.sum()) <= 1e-12 * m0


def test_momentum_gain_equals_body_force():
    rng = np.random.default_rng(4)
    shape = (4, 5, 6)
    g = np.array([2e-5, -1e-5, 3e-6])
    s = Sim(_box(6, 5, 4, [P] * 6, 0.75, body_force=g.tolist()),
            rho0=1 + 0.01 * rng.standard_normal(shape), u0=0.01 * rng.standard_normal((3,) + shape))
    N = 6 * 5 * 4

    def total_momentum():
        f = L.stream(s.S, s.bc, s.u_in, s.rho_out)
        return L.moments(f)[1].reshape(3, -1).sum(1)

    p0 = total_momentum()
    s.run(5)
    np.testing.assert_allclose(total_momentum() - p0, 5 * N * g, rtol=1e-9, atol=1e-15)


def _poiseuille(tau, ny, steps):
    g = 1e-6
    nu = (tau - 0.5) / 3
    y = np.arange(ny)
    exact = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    u0 = np.zeros((3, 2, ny, 3))
    u0[0] = exact[None, :, None]
    s = Sim(_box(3, ny, 2, [P, P, Wl, Wl, P, P], tau, body_force=[g, 0, 0]), u0=u0)
    s.run(steps)
    rho, u = s.fields()
    return u[0, 0, :, 0], exact, g, nu


def test_poiseuille_exact_at_magic_tau():
    # half-way bounce-back makes BGK Poiseuille flow exact when
    # (tau - 1/2)^2 = 3/16 (walls exactly half-way between nodes)
    tau = 0.5 + math.sqrt(3.0) / 4.0
    u, exact, g, nu = _poiseuille(tau, 8, 1500)
    np.testing.assert_allclose(u, exact, rtol=1e-9)


def test_poiseuille_interior_curvature():
    # at any tau the steady discrete profile has u[j+1] - 2u[j] + u[j-1] = -g/nu
    u, exact, g, nu = _poiseuille(0.8, 8, 2500)
    d2 = u[2:] - 2 * u[1:-1] + u[:-2]
    np.testing.assert_allclose(d2, -g / nu, rtol=1e-6)


def _tgv_rate(n, tau, steps):
    u0v = 1e-3
    k = 2 * np.pi / n
    x = np.arange(n)
    yy, xx = np.meshgrid(x, x, indexing="ij")
    u0 = np.zeros((3, 1, n, n))
    u0[0, 0] = u0v * np.sin(k * xx) * np.cos(k * yy)
    u0[1, 0] = -u0v * np.cos(k * xx) * np.sin(k * yy)
    s = Sim(_box(n, n, 1, [P] * 6, tau), u0=u0)
    e = []
    for _ in range(steps):
        s.step()
        rho, u = s.fields()
        e.append(0.5 * (u * u).sum())
    e = np.array(e)
    t = np.arange(1, steps + 1)
    half = steps // 2
    rate = -np.polyfit(t[half:], np.log(e[half:]), 1)[0]
    nu = (tau - 0.5) / 3
    return rate, 4 * nu * k * k


def test_taylor_green_decay_rate_and_convergence():
    # 2D Taylor-Green vortex: kinetic energy decays as exp(-4 nu k^2 t),
    # nu = (tau - 1/2)/3 (Eq. 3).  The relative rate error falls ~4x per
    # doubling of resolution at fixed tau.
    tau = 0.8
    r16, e16 = _tgv_rate(16, tau, 60)
    r32, e32 = _tgv_rate(32, tau, 240)
    err16 = abs(r16 / e16 - 1)
    err32 = abs(r32 / e32 - 1)
    assert err32 < 5e-3
    assert err16 / err32 > 3.0


def test_periodic_translation_invariance():
    rng = np.random.default_rng(5)
    shape = (4, 5, 6)
    rho0 = 1 + 0.01 * rng.standard_normal(shape)
    u0 = 0.02 * rng.standard_normal((3,) + shape)
    bc = [P, P, Wl, Wl, P, P]
    a = Sim(_box(6, 5, 4, bc, 0.7), rho0=rho0, u0=u0)
    b = Sim(_box(6, 5, 4, bc, 0.7), rho0=np.roll(rho0, (1, 2), axis=(0, 2)),
            u0=np.roll(u0, (1, 2), axis=(1, 3)))
    a.run(5)
    b.run(5)
    np.testing.assert_allclose(np.roll(a.S, (1, 2), axis=(1, 3)), b.S, atol=1e-15)


def _zh_state(seed, shape=(6, 7, 9)):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    rho = 1 + 0.01 * rng.standard_normal(shape)
    u = 0.03 * rng.standard_normal((3,) + shape)
    S = L.equilibrium(rho, u) + 1e-3 * rng.standard_normal((19,) + shape) * L.W[:, None, None, None]
    return S


@pytest.mark.parametrize("walls", [False, True])
def test_zou_he_faces_impose_velocity_and_density(walls):
    """Zou-He faces (Sec. 3.1): after streaming, a velocity-face cell carries
    exactly the prescribed velocity, a pressure-face cell exactly the
    prescribed density with zero transverse momentum, and the normal
    population obeys non-equilibrium bounce-back, f_n - f_n^eq equal for the
    entering and the leaving one.  Cells whose entering links touch a wall
    keep the equilibrium-ghost values."""
    S = _zh_state(3)
    yb = L.WALL if walls else L.PERIODIC
    bc = [L.ZH_VELOCITY, L.ZH_PRESSURE, yb, yb, L.PERIODIC, L.PERIODIC]
    u_in = np.array([0.04, -0.01, 0.015])
    f = L.stream(S, bc, u_in, 1.02)
    ys = slice(1, -1) if walls else slice(None)
    rho, mom = L.moments(f)
    # velocity face, x = 0
    r0, m0 = rho[:, ys, 0], mom[:, :, ys, 0]
    assert np.allclose(m0 / r0[None], u_in[:, None, None], rtol=0, atol=1e-14)
    feq = L.equilibrium(r0, np.broadcast_to(u_in[:, None, None], (3,) + r0.shape))
    assert np.allclose(f[1][:, ys, 0] - feq[1], f[2][:, ys, 0] - feq[2], rtol=0, atol=1e-15)
    # pressure face, x = nx - 1
    r1, m1 = rho[:, ys, -1], mom[:, :, ys, -1]
    assert np.allclose(r1, 1.02, rtol=0, atol=1e-14)
    assert np.allclose(m1[1:], 0.0, atol=1e-15)
    u1 = m1 / r1[None]
    feq = L.equilibrium(r1, u1)
    assert np.allclose(f[2][:, ys, -1] - feq[2], f[1][:, ys, -1] - feq[1], rtol=0, atol=1e-15)
    if walls:
        g = L.stream(S, [L.VELOCITY, L.PRESSURE, yb, yb, L.PERIODIC, L.PERIODIC], u_in, 1.02)
        for yy in (0, -1):
            assert np.array_equal(f[:, :, yy, :], g[:, :, yy, :])
    # nothing but the two faces changes
    g = L.stream(S, [L.VELOCITY, L.PRESSURE, yb, yb, L.PERIODIC, L.PERIODIC], u_in, 1.02)
    assert np.array_equal(f[:, :, :, 1:-1], g[:, :, :, 1:-1])


def test_zou_he_uniform_flow_is_a_fixed_point():
    """Uniform flow at the inlet velocity with rho = rho_out stays exactly
    uniform through Zou-He inlet and outlet (periodic y, z)."""
    shape = (4, 5, 8)
    u_in = np.array([0.05, 0.0, 0.0])
    u = np.broadcast_to(u_in[:, None, None, None], (3,) + shape).copy()
    S = L.equilibrium(np.ones(shape), u)
    bc = [L.ZH_VELOCITY, L.ZH_PRESSURE, L.PERIODIC, L.PERIODIC, L.PERIODIC, L.PERIODIC]
    for _ in range(5):
        f = L.stream(S, bc, u_in, 1.0)
        rho, mom = L.moments(f)
        S = L.collide(f, rho, mom / rho, np.zeros((3,) + shape), 0.8)
    assert np.allclose(S, L.equilibrium(np.ones(shape), u), rtol=0, atol=1e-15)


@pytest.mark.parametrize("backend", ["numpy", "c"])
def test_inlet_outlet_half_range_mass_flux(backend):
    """Mass entering through the equilibrium faces (Sec. 2.1), against the
    half-range moments of the equilibrium, worked out by hand for D3Q19:
    over the five populations with c_x = +1, sum w_i [1 + 3 c.u + 4.5 (c.u)^2
    - 1.5 u.u] = (1 + 3 u_x + 3 u_x^2) / 6 for any u_y, u_z, and over c_x = -1
    it is (1 - 3 u_x + 3 u_x^2) / 6.  So after streaming, the populations
    entering a velocity-inlet cell sum to rho_b (1 + 3 U + 3 U^2) / 6 with
    rho_b the density of that boundary cell, and those entering a
    pressure-outlet cell sum to rho_out (1 - 3 u_b + 3 u_b^2) / 6 with u_b the
    x velocity of the boundary cell.  The state varies along x only (y, z
    periodic), with density and velocity different in the neighbouring
    columns, so a ghost taken from any other cell fails."""
    lat = L if backend == "numpy" else __import__("oracle.clattice", fromlist=["x"])
    nz, ny, nx = 3, 4, 7
    x = np.arange(nx)
    rho = np.broadcast_to(1.0 + 0.02 * np.sin(1.3 * x + 0.4), (nz, ny, nx)).copy()
    u = np.zeros((3, nz, ny, nx))
    u[0] = 0.03 + 0.02 * np.cos(0.9 * x)
    u[1] = 0.01 * np.sin(0.7 * x)
    u[2] = -0.015 * np.cos(0.5 * x)
    rng = np.random.default_rng(8)
    neq = 1e-3 * rng.standard_normal((19, nx)) * L.W[:, None]
    # a non-equilibrium part with zero mass and momentum keeps rho, u of S
    A = np.vstack([np.ones(19), L.C.T.astype(float)])          # (4, 19)
    neq = neq - A.T @ np.linalg.solve(A @ A.T, A @ neq)
    S = L.equilibrium(rho, u) + neq[:, None, None, :]
    rS, mS = L.moments(S)
    np.testing.assert_allclose(rS, rho, atol=1e-15)
    U_in, rho_out = 0.045, 1.013
    f = lat.stream(S, [V, PR, P, P, P, P], [U_in, 0.02, -0.01], rho_out)
    inl = f[L.C[:, 0] == 1][:, :, :, 0].sum(axis=0)
    np.testing.assert_allclose(inl, rho[0, 0, 0] * (1 + 3 * U_in + 3 * U_in ** 2) / 6, rtol=1e-14)
    ub = mS[0, 0, 0, nx - 1] / rS[0, 0, nx - 1]
    out = f[L.C[:, 0] == -1][:, :, :, nx - 1].sum(axis=0)
    np.testing.assert_allclose(out, rho_out * (1 - 3 * ub + 3 * ub ** 2) / 6, rtol=1e-14)
    # and the neighbouring column differs, so the pin separates the cells
    assert abs(rho[0, 0, 1] - rho[0, 0, 0]) > 1e-3
    assert abs(mS[0, 0, 0, nx - 2] / rS[0, 0, nx - 2] - ub) > 1e-3
