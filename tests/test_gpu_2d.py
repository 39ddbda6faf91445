"""The paper's 2D scheme on the GPU: the library on one periodic layer
(nz = 1), which is D2Q9 exactly (pinned on the CPU against an independent
D2Q9 oracle), compared with that D2Q9 oracle for both of the paper's moving
cases: the figure-eight hovering stroke (Sec. 3.2) and clap & fling
(Sec. 3.3), u and C_L / C_T per step."""
import sys

import numpy as np
import pytest

import workloads as WL
from tests.helpers import coeff_errors, gpu_solver, l2rel

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", ["figure_eight", "clap_fling"])
def test_2d_against_d2q9_oracle(case):
    from oracle import d2q9 as D2
    from oracle import params

    if case == "figure_eight":
        bx, wg, ph = WL.figure_eight_case(nx=96, ny=96, nz=1)
        t0, steps = 300, 150
    else:
        bx, wg, ph = WL.clap_fling_case(nx=128, ny=96, nz=1, chord=12.0, re=100.0, j=0.5, f=0.25)
        t0, steps = 200, 150
    _say("2D", case, bx["nx"], "x", bx["ny"], "from", t0, "for", steps)
    ob, ow = params.complete_case(bx, wg, ph)
    u0 = WL.velocity_noise((1, bx["ny"], bx["nx"]), 8)
    u0[2] = 0.0
    u_gpu = u0.copy()
    u_ora = u0[:2, 0].copy()
    u_ora[0] += ob["u_in"][0]
    gpu = gpu_solver(bx, wg, ph, u0=u_gpu, step0=t0)   # adds the inflow itself for clap & fling
    ora = D2.Sim2D(ob, ow, u0=u_ora)
    ora.n = t0
    gpu.step(steps)
    ora.run(steps)
    rho_o, u_o = ora.fields()
    u_g = gpu.fields("u")
    err = l2rel(u_g[:2, 0], u_o)
    print("L2 rel u", err, "max |u_z|", np.abs(u_g[2]).max())
    assert err <= 1e-5
    assert np.abs(u_g[2]).max() <= 1e-6 * np.abs(u_o).max()
    d = coeff_errors(gpu.forces(t0, steps), ora.forces())
    print("coefficients max rel", d)
    assert max(d.values()) <= 1e-3
    gpu.close()
