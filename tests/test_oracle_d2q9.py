"""The paper's 2D scheme (D2Q9, Eq. 5) against the D3Q19 oracle on one
periodic layer: summing the D3Q19 populations that share (c_x, c_y) gives
the D2Q9 weights, equilibrium, Guo term and streaming, so the two
independent codes must agree step by step -- lattice only, with every face
kind, and with moving foils (interpolation, solve, spreading, forces).
This pins the 2D mode of the library (nz = 1, periodic z)."""
import math

import numpy as np
import pytest

import workloads as WL
from oracle import d2q9 as D2
from oracle import lattice as L
from oracle import params
from oracle.sim import Sim


def test_d2q9_tables_are_the_projection_of_d3q19():
    assert D2.W.sum() == pytest.approx(1.0, abs=1e-16)
    for i in range(D2.Q):
        sel = (L.C[:, 0] == D2.C[i, 0]) & (L.C[:, 1] == D2.C[i, 1])
        assert L.W[sel].sum() == pytest.approx(D2.W[i], abs=1e-16)
    # second moment c_s^2 = 1/3, fourth-order isotropy
    assert np.allclose(np.einsum("q,qa,qb->ab", D2.W, D2.C, D2.C), np.eye(2) / 3.0, atol=1e-16)


def _project(S3):
    """(19, 1, ny, nx) -> (9, ny, nx): sum over the populations of equal (c_x, c_y)."""
    out = np.zeros((D2.Q,) + S3.shape[2:])
    for i in range(D2.Q):
        sel = (L.C[:, 0] == D2.C[i, 0]) & (L.C[:, 1] == D2.C[i, 1])
        out[i] = S3[sel, 0].sum(axis=0)
    return out


CASES = [
    ("channel_force", [L.PERIODIC, L.PERIODIC, L.WALL, L.WALL], dict(body_force=[2e-5, 0, 0])),
    ("inlet_outlet", [L.VELOCITY, L.PRESSURE, L.WALL, L.WALL], dict(u_in=[0.03, 0.004, 0.0])),
    ("zou_he", [L.ZH_VELOCITY, L.ZH_PRESSURE, L.WALL, L.WALL], dict(u_in=[0.03, 0.004, 0.0], rho_out=1.01)),
    ("zou_he_periodic", [L.ZH_VELOCITY, L.ZH_PRESSURE, L.PERIODIC, L.PERIODIC], dict(u_in=[0.02, -0.003, 0.0])),
    ("closed", [L.WALL, L.WALL, L.WALL, L.WALL], {}),
]


@pytest.mark.parametrize("name,bc,extra", CASES, ids=[c[0] for c in CASES])
def test_lattice_2d_equals_d3q19_on_one_layer(name, bc, extra):
    nx, ny = 23, 14
    rng = np.random.default_rng(5)
    rho0 = 1 + 0.01 * rng.standard_normal((ny, nx))
    u0 = 0.03 * rng.standard_normal((2, ny, nx))
    bx = dict(nx=nx, ny=ny, nz=1, bc=bc + [L.PERIODIC, L.PERIODIC], tau=0.7, u_in=[0, 0, 0],
              rho_out=1.0, body_force=[0, 0, 0])
    bx.update(extra)
    s3 = Sim(bx, [], rho0=rho0[None], u0=np.concatenate([u0, np.zeros((1, ny, nx))])[:, None])
    s2 = D2.Sim2D(bx, [], rho0=rho0, u0=u0)
    assert np.allclose(_project(s3.S), s2.S, atol=1e-16)
    s3.run(25)
    s2.run(25)
    assert np.allclose(_project(s3.S), s2.S, rtol=0, atol=2e-15)
    r3, u3 = s3.fields()
    r2, u2 = s2.fields()
    assert np.allclose(u3[:2, 0], u2, rtol=0, atol=1e-15)
    assert np.allclose(u3[2], 0.0, atol=1e-17)


@pytest.mark.parametrize("case", ["figure_eight", "clap_fling"])
def test_ibm_2d_equals_d3q19_on_one_layer(case):
    """Moving foils: the span factor of one periodic layer is exactly 1, so
    the 3D minimum-norm solve reduces to the 2D perimeter solve."""
    if case == "figure_eight":
        bx, wg, ph = WL.figure_eight_case(nz=1)
        t0 = 200
    else:
        bx, wg, ph = WL.clap_fling_case(nx=64, ny=48, nz=1, chord=8.0, re=100.0, j=0.5, f=0.25)
        t0 = 150
    ob, ow = params.complete_case(bx, wg, ph)
    ny, nx = ob["ny"], ob["nx"]
    u0 = WL.velocity_noise((1, ny, nx), 3)
    u0[0] += ob["u_in"][0]
    u0[2] = 0.0                      # a 2D flow: no span velocity
    s3 = Sim(ob, ow, u0=u0)
    s2 = D2.Sim2D(ob, ow, u0=u0[:2, 0])
    s3.n = s2.n = t0
    s3.run(12)
    s2.run(12)
    r3, u3 = s3.fields()
    r2, u2 = s2.fields()
    assert np.allclose(u3[:2, 0], u2, rtol=0, atol=1e-13)
    f3, f2 = s3.forces(), s2.forces()
    scale = np.abs(f2[:, :, :2]).max()
    assert np.allclose(f3[:, :, [0, 1, 3]], f2[:, :, [0, 1, 3]], rtol=0, atol=1e-10 * scale)
