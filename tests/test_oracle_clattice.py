"""Pins of the oracle's C lattice (oracle/clattice.c, the same operations
as oracle/lattice.py in plain C with OpenMP, used for long runs on large
boxes).

It is checked two ways: against lattice.py on random states for every
combination of face kinds (streaming, moments, collision, equilibrium) and
on whole IB-LBM runs with moving foils; and on its own against the closed
forms the lattice pins use (mass conservation in closed boxes, uniform flow
through inlet and outlet as a fixed point, momentum gain equal to the body
force, Poiseuille flow exact at (tau - 1/2)^2 = 3/16, Zou-He faces imposing
their velocity and density).
"""
import math

import numpy as np
import pytest

import workloads as WL
from oracle import clattice as CL
from oracle import lattice as L
from oracle import params
from oracle.sim import Sim
from tests.helpers import clap_fling, plate

P, Wl, V, PR, ZV, ZP = 0, 1, 2, 3, 4, 5

BCS = [[V, PR, Wl, Wl, P, P], [PR, V, P, P, Wl, Wl], [ZV, ZP, Wl, Wl, P, P], [ZP, ZV, P, P, P, P],
       [Wl] * 6, [P] * 6, [V, PR, P, P, P, P], [ZV, PR, Wl, Wl, Wl, Wl], [P, P, Wl, Wl, P, P]]


def _box(nx, ny, nz, bc, tau, **kw):
    d = dict(nx=nx, ny=ny, nz=nz, bc=bc, tau=tau, u_in=[0, 0, 0], rho_out=1.0,
             body_force=[0, 0, 0], u_ref=1.0, area_ref=1.0)
    d.update(kw)
    return d


@pytest.mark.parametrize("bc", BCS)
def test_operations_equal_lattice_py(bc):
    rng = np.random.default_rng(11)
    nz, ny, nx = 5, 6, 7
    rho = 1 + 0.05 * rng.standard_normal((nz, ny, nx))
    u = 0.05 * rng.standard_normal((3, nz, ny, nx))
    S = L.equilibrium(rho, u) + 1e-3 * rng.standard_normal((19, nz, ny, nx))
    u_in = [0.03, 0.01, -0.02]
    f = L.stream(S, bc, u_in, 1.02)
    np.testing.assert_allclose(CL.stream(S, bc, u_in, 1.02), f, rtol=0, atol=1e-15)
    r, m = L.moments(f)
    rc, mc = CL.moments(f)
    np.testing.assert_allclose(rc, r, rtol=0, atol=1e-15)
    np.testing.assert_allclose(mc, m, rtol=0, atol=1e-15)
    F = 1e-3 * rng.standard_normal((3, nz, ny, nx))
    np.testing.assert_allclose(CL.collide(f, r, m / r, F, 0.57), L.collide(f, r, m / r, F, 0.57),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(CL.equilibrium(rho, u), L.equilibrium(rho, u), rtol=0, atol=1e-16)


@pytest.mark.parametrize("case", ["plate", "clap_fling", "figure_eight"])
def test_ibm_runs_equal_lattice_py(case):
    if case == "plate":
        bx, wg, ph, u0 = plate(nz=4, seed=1)
        steps = 25
    elif case == "clap_fling":
        bx, wg, ph, u0 = clap_fling(seed=2, nx=64, ny=48, nz=4, chord=8.0, re=100.0, j=0.5, f=0.25)
        steps = 40
    else:
        bx, wg, ph = WL.figure_eight_case(nx=48, ny=48, nz=2, chord=10.0)
        u0 = WL.velocity_noise((2, 48, 48), 3)
        steps = 30
    ob, ow = params.complete_case(bx, wg, ph)
    if ph["kind"] == "clap_fling":
        u0 = u0.copy()
        u0[0] += ob["u_in"][0]
    a = Sim(ob, ow, u0=u0)
    b = Sim(ob, ow, u0=u0, lattice="c")
    a.run(steps)
    b.run(steps)
    scale = np.abs(a.S).max()
    assert np.abs(a.S - b.S).max() <= 1e-13 * scale
    fa, fb = a.forces(), b.forces()
    assert np.abs(fa - fb).max() <= 1e-11 * np.abs(fa).max()


@pytest.mark.parametrize("bc", [[P] * 6, [Wl, Wl, Wl, Wl, P, P], [Wl] * 6])
def test_mass_conservation_closed_box(bc):
    rng = np.random.default_rng(3)
    shape = (6, 7, 8)
    rho0 = 1 + 0.01 * rng.standard_normal(shape)
    u0 = 0.02 * rng.standard_normal((3,) + shape)
    s = Sim(_box(8, 7, 6, bc, 0.62), rho0=rho0, u0=u0, lattice="c")
    m0 = s.mass()
    s.run(60)
    assert abs(s.mass() - m0) <= 1e-13 * m0
    assert abs(m0 - rho0.sum()) <= 1e-12 * m0


@pytest.mark.parametrize("bc", [[V, PR, P, P, P, P], [ZV, ZP, P, P, P, P]])
def test_uniform_flow_is_fixed_point_with_inlet_outlet(bc):
    U = 0.04
    u0 = np.zeros((3, 4, 6, 9))
    u0[0] = U
    s = Sim(_box(9, 6, 4, bc, 0.7, u_in=[U, 0, 0]), u0=u0, lattice="c")
    S0 = s.S.copy()
    s.run(4)
    np.testing.assert_allclose(s.S, S0, rtol=0, atol=1e-15)


def test_momentum_gain_equals_body_force():
    rng = np.random.default_rng(4)
    shape = (4, 5, 6)
    g = np.array([2e-5, -1e-5, 3e-6])
    s = Sim(_box(6, 5, 4, [P] * 6, 0.75, body_force=g.tolist()),
            rho0=1 + 0.01 * rng.standard_normal(shape), u0=0.01 * rng.standard_normal((3,) + shape),
            lattice="c")
    N = 6 * 5 * 4

    def total_momentum():
        f = CL.stream(s.S, s.bc, s.u_in, s.rho_out)
        return CL.moments(f)[1].reshape(3, -1).sum(1)

    p0 = total_momentum()
    s.run(5)
    np.testing.assert_allclose(total_momentum() - p0, 5 * N * g, rtol=1e-9, atol=1e-15)


def test_poiseuille_exact_at_magic_tau():
    tau = 0.5 + math.sqrt(3.0) / 4.0
    g = 1e-6
    nu = (tau - 0.5) / 3
    ny = 8
    y = np.arange(ny)
    exact = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    u0 = np.zeros((3, 2, ny, 3))
    u0[0] = exact[None, :, None]
    s = Sim(_box(3, ny, 2, [P, P, Wl, Wl, P, P], tau, body_force=[g, 0, 0]), u0=u0, lattice="c")
    s.run(1500)
    _, u = s.fields()
    np.testing.assert_allclose(u[0, 0, :, 0], exact, rtol=1e-9)


def test_zou_he_faces_impose_velocity_and_density():
    rng = np.random.default_rng(3)
    shape = (6, 7, 9)
    rho = 1 + 0.01 * rng.standard_normal(shape)
    u = 0.03 * rng.standard_normal((3,) + shape)
    S = L.equilibrium(rho, u) + 1e-3 * rng.standard_normal((19,) + shape) * L.W[:, None, None, None]
    u_in = np.array([0.04, -0.01, 0.015])
    f = CL.stream(S, [ZV, ZP, P, P, P, P], u_in, 1.02)
    r, m = CL.moments(f)
    assert np.allclose(m[:, :, :, 0] / r[None, :, :, 0], u_in[:, None, None], rtol=0, atol=1e-14)
    assert np.allclose(r[:, :, -1], 1.02, rtol=0, atol=1e-14)
    assert np.allclose(m[1:, :, :, -1], 0.0, atol=1e-15)
