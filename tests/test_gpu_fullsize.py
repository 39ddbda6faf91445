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


def test_large_config_properties():
    """The largest workload, 512x384x384 with two c = 40 wings (2 x 84 x 384
    markers), too large for the oracle: properties that hold at any size.
    Started at rest (plus the free stream) from mid-stroke, the pair stays
    mirror-symmetric, so F_x agree and F_y are opposite for the two wings at
    every step; and the FP16 run follows the FP32 run within the FP16
    storage bar over the whole box."""
    _say("clap & fling 512x384x384, c=40, 10 steps from step 37, fp32 and fp16")
    bx, wg, ph = WL.clap_fling_case(nx=512, ny=384, nz=384, chord=40.0, re=150.0, j=0.01, f=0.25)
    u0 = np.zeros((3, bx["nz"], bx["ny"], bx["nx"]))
    runs = {}
    for storage in ("fp32", "fp16"):
        gpu = gpu_solver(bx, wg, ph, u0=u0, step0=37, storage=storage)
        gpu.step(10)
        runs[storage] = (gpu.forces(37, 10), gpu.fields("u"))
        gpu.close()
    h, u32 = runs["fp32"]
    assert np.isfinite(h).all() and np.isfinite(u32).all()
    scale = np.abs(h[:, :, :2]).max()
    sym_x = np.abs(h[:, 0, 0] - h[:, 1, 0]).max() / scale
    sym_y = np.abs(h[:, 0, 1] + h[:, 1, 1]).max() / scale
    e16 = l2rel(runs["fp16"][1], u32)
    print(f"[large] mirror Fx {sym_x:.2e} Fy {sym_y:.2e}; fp16 vs fp32 L2 rel u {e16:.2e}", flush=True)
    assert sym_x <= 1e-4 and sym_y <= 1e-4
    assert e16 <= 1e-3
