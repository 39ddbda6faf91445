"""Parity at the benchmark's own size, in the configuration bench.py times:
clap & fling 256x192x192, two wings (c = 20, 2 x 42 x 192 markers),
Re = 100, J = 0.01, f = 0.25, seeded initial noise.  The FP64 oracle runs
the same eight steps on the whole box (about 30 s on the host); the GPU result
is compared cell by cell (u over all 9.4M cells) and per step (C_L, C_T of
both foils), for FP32 (bars 1e-5 / 1e-3) and for FP16 and BF16 (their
storage bars: u 1e-3 / 8e-3, coefficients 1e-3 / 3e-2)."""
import sys

import numpy as np
import pytest

import workloads as WL
from tests.helpers import gpu_solver, l2rel, oracle_sim

pytestmark = pytest.mark.gpu

STEPS = 8
_ORA = {}


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _case():
    bx, wg, ph = WL.clap_fling_case(nx=256, ny=192, nz=192, chord=20.0, re=100.0, j=0.01, f=0.25)
    u0 = WL.velocity_noise((bx["nz"], bx["ny"], bx["nx"]), 0)
    return bx, wg, ph, u0


def _oracle():
    if not _ORA:
        bx, wg, ph, u0 = _case()
        ora = oracle_sim(bx, wg, ph, u0=u0)
        ora.run(STEPS)
        _ORA["u"] = ora.fields()[1]
        _ORA["f"] = ora.forces()
    return _ORA["u"], _ORA["f"]


@pytest.mark.parametrize("storage,bar_u,bar_c", [("fp32", 1e-5, 1e-3), ("fp16", 1e-3, 1e-3), ("bf16", 8e-3, 3e-2)])
def test_clap_fling_full_size(storage, bar_u, bar_c):
    _say("clap & fling 256x192x192, full size,", STEPS, "steps,", storage)
    bx, wg, ph, u0 = _case()
    gpu = gpu_solver(bx, wg, ph, u0=u0, storage=storage)
    gpu.step(STEPS)
    u_g = gpu.fields("u")
    f_g = gpu.forces(0, STEPS)
    gpu.close()
    u_o, f_o = _oracle()
    e = l2rel(u_g, u_o)
    dc = {}
    for k, name in ((4, "cl"), (5, "ct")):
        dc[name] = max(np.abs(f_g[:, w, k] - f_o[:, w, k]).max() / np.abs(f_o[:, w, k]).max()
                       for w in range(2))
    print(f"[fullsize] {storage} L2 rel u {e:.3e} C_L {dc['cl']:.3e} C_T {dc['ct']:.3e}", flush=True)
    assert e <= bar_u
    assert dc["cl"] <= bar_c
    assert dc["ct"] <= bar_c
