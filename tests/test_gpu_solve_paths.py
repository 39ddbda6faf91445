"""Oracle parity on small boxes that reach the code paths of the
512x384x384 workload (two c = 40 foils, 384 span layers):

* a span of 384 layers: the per-marker interpolation and span-solve block
  then runs with 256 threads and two parts of the span range (up to about
  330 layers it runs 512 threads and eight parts);
* chord 40: 84 perimeter markers per layer, so the 84 x 84 perimeter
  inverse, its window of factors and the layer kernel's larger node box;
* chord 48: over 96 perimeter markers, the largest register tile of the
  perimeter factor.

Both cases compare u (global L2 and element-wise on the marker supports),
every force/moment column per step and the marker quantities of the last
step (interpolated density, right-hand side B and du_B of Eq. 19) with the
FP64 oracle, in FP32 storage, with the bars of the plate workload.  The
oracle runs its C lattice here (same results as lattice.py to rounding)."""
import math
import sys

import numpy as np
import pytest

from tests.helpers import clap_fling, coeff_errors, gpu_solver, l2rel, node_box_error, oracle_sim

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _run(case, step0, steps):
    from oracle import params
    from oracle.sim import Sim

    bx, wg, ph, u0 = clap_fling(**case)
    gpu = gpu_solver(bx, wg, ph, u0=u0, step0=step0)
    ob, ow = params.complete_case(bx, wg, ph)
    u = u0.copy()
    u[0] += ob["u_in"][0]
    ora = Sim(ob, ow, u0=u, lattice="c")
    ora.n = step0
    gpu.step(steps)
    ora.run(steps)
    return gpu, ora


def _check(gpu, ora, step0, steps):
    rho_o, u_o = ora.fields()
    u_g = gpu.fields("u")
    err = l2rel(u_g, u_o)
    eb = node_box_error(u_g, u_o, ora.last["nodes"])
    d = coeff_errors(gpu.forces(step0, steps), ora.forces())
    Lr = ora.last
    e_rb = float(np.abs(gpu.markers("rhoB") - Lr["rhoB"]).max())
    e_b = float(np.abs(gpu.markers("B") - Lr["B"]).max() / np.abs(Lr["B"]).max())
    duB_o = Lr["duB"].T
    e_du = float(np.abs(gpu.markers("duB") - duB_o).max() / np.abs(duB_o).max())
    print(f"[paths] L2 u {err:.3e} node-box {eb:.3e} rhoB {e_rb:.3e} B {e_b:.3e} duB {e_du:.3e} "
          f"coefficients {d}", flush=True)
    assert err <= 1e-5
    assert eb <= 1e-5
    assert max(d.values()) <= 1e-3
    assert e_rb <= 2e-6
    assert e_b <= 1e-4
    assert e_du <= 1e-4


def test_span_of_384_layers():
    case = dict(seed=9, nx=64, ny=48, nz=384, chord=8.0, re=100.0, j=0.5, f=0.25)
    _say("clap & fling 64x48x384, c=8 (256-thread span solve), 12 steps from step 150")
    gpu, ora = _run(case, 150, 12)
    _check(gpu, ora, 150, 12)
    gpu.close()


def test_chord_40_perimeter():
    case = dict(seed=10, nx=128, ny=112, nz=16, chord=40.0, re=150.0, j=0.01, f=0.25)
    from oracle import params
    bx, wg, ph, _ = clap_fling(**case)
    T = params.complete_case(bx, wg, ph)[1][0]["period_steps"]
    t0 = int(T / 8)
    _say("clap & fling 128x112x16, c=40 (84 perimeter markers), 20 steps from step", t0)
    gpu, ora = _run(case, t0, 20)
    assert gpu.markers("dA").size == 2 * 84 * 16
    _check(gpu, ora, t0, 20)
    gpu.close()


def test_chord_48_perimeter():
    """Chord 48: about 101 perimeter markers per layer, past 96, so the
    perimeter factor holds its block in the largest register tile (8 x 8
    entries per thread)."""
    case = dict(seed=11, nx=160, ny=144, nz=8, chord=48.0, re=150.0, j=0.01, f=0.25)
    from oracle import params
    bx, wg, ph, _ = clap_fling(**case)
    T = params.complete_case(bx, wg, ph)[1][0]["period_steps"]
    t0 = int(T / 8)
    _say("clap & fling 160x144x8, c=48 (over 96 perimeter markers), 12 steps from step", t0)
    gpu, ora = _run(case, t0, 12)
    n_p = gpu.markers("dA").size // (2 * 8)
    assert 96 < n_p <= 128, n_p
    _check(gpu, ora, t0, 12)
    gpu.close()
