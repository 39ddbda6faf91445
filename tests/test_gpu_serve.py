"""Served form on the GPU: grouped stepping of several solves at once.

* Alone vs mix: a solve stepped inside a batch (with solves of other sizes,
  parameters, storages, and one that joins later) gives exactly the forces
  and fields it gives alone, across launch-argument windows that start at
  different steps for different solves.  The mix holds a span of 200
  layers (whose span solve runs 512 threads alone) beside one of 384 (256
  threads), so the grouped launch runs the first with fewer threads than
  alone; its sums keep their order.
* The sweep server under an HBM budget that holds two solves at a time:
  every request completes, the budget holds, and a served clap & fling
  request matches the FP64 oracle (C_L within 1e-3 of max|C_L|).
"""
import sys

import numpy as np
import pytest

import workloads as WL
from tests.helpers import clap_fling, coeff_errors, gpu_solver, l2rel, oracle_sim

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _solves():
    """(name, bx, wg, ph, u0, storage, step0) of four different solves."""
    a = clap_fling(seed=6, nx=64, ny=48, nz=8, chord=8.0, re=100.0, j=0.5, f=0.25)
    b = clap_fling(seed=1, nx=64, ny=64, nz=64, chord=8.0, re=75.0, j=0.01, f=0.05)
    c = clap_fling(seed=2, nx=96, ny=80, nz=16, chord=10.0, re=150.0, j=2.0, f=0.25)
    d = clap_fling(seed=3, nx=64, ny=48, nz=200, chord=8.0, re=100.0, j=0.5, f=0.25)
    e = clap_fling(seed=4, nx=64, ny=48, nz=384, chord=8.0, re=150.0, j=0.01, f=0.25)
    tg_bx, tg_r, tg_u, _ = WL.taylor_green_case(32)
    return [
        ("cf64x48x8", a[0], a[1], a[2], a[3], "fp32", 0),
        ("cf64^3", b[0], b[1], b[2], b[3], "fp32", 37),
        ("cf96x80x16_fp16", c[0], c[1], c[2], c[3], "fp16", 5),
        ("tg32", tg_bx, [], None, tg_u, "fp32", 0),
        ("cf64x48x200_span512", d[0], d[1], d[2], d[3], "fp32", 11),
        ("cf64x48x384_span256", e[0], e[1], e[2], e[3], "fp32", 0),
    ]


def _make(case):
    name, bx, wg, ph, u0, storage, step0 = case
    return gpu_solver(bx, wg, ph, u0=u0, storage=storage, step0=step0)


def test_batch_alone_vs_mix_bitwise():
    from paper_2102_01305_amd.solver import step_batch

    cases = _solves()
    total = 150
    alone = []
    for case in cases:
        _say("alone", case[0], total, "steps")
        s = _make(case)
        s.step(total)
        alone.append((s.forces(case[6], total) if case[2] else None, s.fields("u")))
        s.close()
    _say("mix: 0,1 for 20 steps; 0,1,2 for 70; all six for 60; then 2..5 and 3..5 to", total)
    ss = [_make(c) for c in cases]
    step_batch(ss[:2], 20)
    step_batch(ss[:3], 70)
    step_batch(ss, 60)                 # 0 and 1 reach 150
    step_batch(ss[2:], 20)             # 2 reaches 150
    step_batch(ss[3:], 70)             # 3, 4 and 5 reach 150
    for case, s, (fa, ua) in zip(cases, ss, alone):
        assert s.step_count == case[6] + total
        fm = s.forces(case[6], total) if case[2] else None
        um = s.fields("u")
        if fa is not None:
            assert np.array_equal(fa, fm), case[0]
        assert np.array_equal(ua, um), case[0]
        s.close()


def test_batch_rejects_bad_handle_lists():
    from paper_2102_01305_amd import _lib as L
    from paper_2102_01305_amd.solver import step_batch

    cases = _solves()
    s = _make(cases[0])
    with pytest.raises(L.IbmlbmError):
        step_batch([s, s], 1)
    s.close()


def test_server_budget_and_oracle():
    import torch

    from paper_2102_01305_amd.serve import SweepRequest, SweepServer, summarize
    from paper_2102_01305_amd.solver import complete_case, workspace_bytes

    reqs = []
    specs = [(64, 48, 8, 8.0, 100.0, 0.5, 0.25, 6), (64, 64, 64, 8.0, 75.0, 0.01, 0.05, 1),
             (64, 48, 8, 8.0, 150.0, 2.0, 0.25, 3), (96, 80, 16, 10.0, 100.0, 0.01, 0.25, 4),
             (64, 64, 64, 8.0, 100.0, 0.001, 0.25, 5)]
    for i, (nx, ny, nz, c, re, j, f, seed) in enumerate(specs):
        bx, wg, ph, u0 = clap_fling(seed=seed, nx=nx, ny=ny, nz=nz, chord=c, re=re, j=j, f=f)
        gb, gw = complete_case(bx, wg, ph)
        u = u0.copy()
        u[0] += gb["u_in"][0]
        reqs.append(SweepRequest(rid=i, box=gb, wings=gw, steps=80 + 20 * i, arrival=0.0, u0=u))
    big = max(workspace_bytes(r.box, r.wings, history_steps=r.steps) for r in reqs)
    budget = int(2.2 * big)
    _say("server: 5 requests, budget", budget)
    srv = SweepServer(hbm_budget=budget, chunk=16)
    res = srv.run(reqs)
    torch.cuda.synchronize()
    assert all(r.error is None for r in res)
    assert srv.peak_bytes <= budget
    s = summarize(res)
    print("[serve]", s, "batch sizes", sorted(set(srv.batch_sizes)), flush=True)
    assert s["completed"] == 5
    assert max(srv.batch_sizes) >= 2          # solves did share the device
    # request 0 against the oracle
    bx, wg, ph, u0 = clap_fling(seed=6, nx=64, ny=48, nz=8, chord=8.0, re=100.0, j=0.5, f=0.25)
    ora = oracle_sim(bx, wg, ph, u0=u0)
    ora.run(80)
    fo = ora.forces()
    fg = res[0].forces
    d = coeff_errors(fg, fo)
    print("[serve] served request 0, max|dC|/max|C|", d, flush=True)
    assert max(d.values()) <= 1e-3
