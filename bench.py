"""Throughput of the D3Q19 BGK + implicit-IBM time step on one MI355X.

A step is one pass of the whole hot path over the lattice: marker
kinematics, delta interpolation, the no-slip solve, spreading, the fused
collide-stream with Guo forcing and the force/coefficient reduction.  The
default workload is the clap & fling pair (chord 20, aspect 5) in a
256x192x192 box at Re = 100, J = 0.01, f = 0.25, FP32 storage, synthetic
seeded initial noise.  Prints one JSON line; the default run adds, under
"variants", the same measurement for FP16 and BF16 storage, the 512x384x384
solve (FP32, FP16) and the 256^3 Taylor-Green lattice (FP16).

    python bench.py [--steps K] [--warmup W]
                    [--workload cf|large|plate|tgv|fig8_2d|cylinder|periodic:NXxNYxNZ]
                    [--storage fp32|fp16|bf16] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as WL  # noqa: E402

METRIC = "MLUPS (D3Q19+IBM) & fraction of HBM roofline; sweep p50/p99 latency"
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak


def workload(name):
    if name == "cf":
        bx, wg, ph = WL.clap_fling_case(nx=256, ny=192, nz=192, chord=20.0, re=100.0, j=0.01, f=0.25)
        return "clap_fling_256x192x192", bx, wg, ph
    if name == "large":
        bx, wg, ph = WL.clap_fling_case(nx=512, ny=384, nz=384, chord=40.0, re=150.0, j=0.01, f=0.25)
        return "clap_fling_512x384x384", bx, wg, ph
    if name == "plate":
        bx, wg, ph = WL.plate_case()
        return "plate_64x32x32", bx, wg, ph
    if name == "fig8_2d":
        # the figure-eight hover in the 2D mode (one periodic layer) at the
        # paper's domain of 50 c x 25 c with c = 20
        bx, wg, ph = WL.figure_eight_case(nx=1000, ny=500, nz=1, chord=20.0)
        return "figure_eight_2d_1000x500", bx, wg, ph
    if name == "cylinder":
        # stationary cylinder between Zou-He velocity and pressure faces
        bx, wg, ph = WL.cylinder_case(nx=256, ny=192, nz=192, d=20.0, re=10.0, u_inf=0.04)
        return "cylinder_zou_he_256x192x192", bx, wg, ph
    if name == "tgv":
        bx, r0, u0, nu = WL.taylor_green_case(256)
        return "taylor_green_256", bx, [], dict(kind="taylor_green", re=100.0, rho0=r0, u0=u0)
    if name.startswith("periodic:"):
        # a fully periodic box of any shape with seeded velocity noise and no
        # foils: the collide alone, for comparing box shapes and footprints
        try:
            nx, ny, nz = (int(v) for v in name.split(":", 1)[1].split("x"))
        except ValueError:
            raise SystemExit(f"periodic workload wants periodic:NXxNYxNZ, got {name}")
        bx = WL.box(nx, ny, nz, [WL.PERIODIC] * 6, 0.6)
        u0 = WL.velocity_noise((nz, ny, nx), 0, amp=1e-2)
        return f"periodic_{nx}x{ny}x{nz}", bx, [], dict(kind="lattice", re=None, rho0=None, u0=u0)
    raise SystemExit(f"unknown workload {name}")


# Sources the collide kernel is compiled from: a traffic figure measured with
# hardware counters holds only while these are unchanged.
COLLIDE_SOURCES = ("paper_2102_01305_amd/csrc/collide.hip", "paper_2102_01305_amd/csrc/lattice_dev.h",
                   "paper_2102_01305_amd/csrc/internal.h")


def collide_source_hash():
    """Hash of the collide sources with comments and blank lines left out,
    so that an edit of the documentation alone keeps a counter figure."""
    import hashlib
    import re

    h = hashlib.sha256()
    for rel in COLLIDE_SOURCES:
        with open(os.path.join(ROOT, rel)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(name, storage):
    """HBM bytes per collide launch from the counter summary under profiles/
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None
    when there is none for this workload or the collide sources changed since."""
    path = os.path.join(ROOT, "profiles", f"k_collide_{name}_{storage}_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and " = " in line:
                k, v = line[2:].split(" = ", 1)
                kv[k.strip()] = v.strip().strip("`")
    if kv.get("collide_source_sha256") != collide_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Bandwidth of a plain device copy (read + write of nbytes), timed with
    events on the stream the copy runs on."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    gbs = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling the HBM byte counters:
    each launch reads and writes `nbytes`."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": reps}))


def initial_velocity(bx, ph, u_inf, seed=0):
    u0 = WL.velocity_noise((bx["nz"], bx["ny"], bx["nx"]), seed)
    u0[0] += u_inf
    return u0


def host_cores():
    """Host cores this process may run on (the machine's CPU share)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_rate(bx, wg, ph, u0, steps, rho0=None, lattice="numpy", threads=1):
    """MLUPS of the FP64 oracle over `steps` whole steps (setup excluded):
    lattice.py (NumPy, single-threaded by construction: element-wise array
    operations) or its C lattice with OpenMP over z-planes on `threads`
    threads; the marker part is NumPy/SciPy either way."""
    from threadpoolctl import threadpool_limits

    from oracle import params
    from oracle.sim import Sim

    if ph["kind"] in ("taylor_green", "lattice"):
        ob, ow = bx, wg
    else:
        ob, ow = params.complete_case(bx, wg, ph)
    if lattice == "c":
        from oracle import clattice
        clattice.set_threads(threads)
    with threadpool_limits(limits=threads):
        s = Sim(ob, ow, rho0=rho0, u0=u0, lattice=lattice)
        t0 = time.perf_counter()
        s.run(steps)
        dt = time.perf_counter() - t0
    n = bx["nx"] * bx["ny"] * bx["nz"]
    return n * steps / dt / 1e6, dt


def cpu_baseline(name, bx, wg, ph, u0, steps, rho0=None):
    """The FP64 oracle on the host: the plain NumPy oracle on one core over
    `steps` steps of the benchmark workload; beside it the oracle with its
    C lattice on every host core over a longer window of the same workload,
    and the NumPy oracle over the whole 200-step plate workload."""
    cores = host_cores()
    v1, t1 = _oracle_rate(bx, wg, ph, u0, steps, rho0)
    out = dict(value=round(v1, 3), unit="MLUPS", cores=1, host_cores=cores, kind="oracle",
               sample=f"{steps} whole step(s) of {name} ({bx['nx']}x{bx['ny']}x{bx['nz']}, every marker), "
                      f"FP64 NumPy oracle on one core, {t1:.1f} s")
    if ph["kind"] not in ("taylor_green", "lattice"):
        va, ta = _oracle_rate(bx, wg, ph, u0, 4 * steps, rho0, lattice="c", threads=cores)
        out["all_cores"] = dict(value=round(va, 3), unit="MLUPS", cores=cores,
                                sample=f"{4 * steps} whole steps of {name}, FP64 oracle with its C lattice "
                                       f"(OpenMP over z-planes) on {cores} threads, {ta:.1f} s")
    pb, pw, pp = WL.plate_case()
    pu = WL.velocity_noise((pb["nz"], pb["ny"], pb["nx"]), 0)
    pu[0] += pp["u_inf"]
    vp, tp = _oracle_rate(pb, pw, pp, pu, 200)
    out["plate_200_steps"] = dict(value=round(vp, 3), unit="MLUPS", cores=1,
                                  sample=f"the 64x32x32 plate workload in full (200 steps), FP64 NumPy oracle "
                                         f"on one core, {tp:.1f} s")
    return out


def serve_bench(budget_bytes, steps, storage="fp32"):
    """The seeded 64-request sweep (Re x J x f x domain) served twice: all
    arriving at once (capacity), then with Poisson arrivals at 0.8 of that
    capacity.  Returns the summaries."""
    import torch

    from paper_2102_01305_amd.serve import SweepRequest, SweepServer, summarize
    from paper_2102_01305_amd.solver import complete_case

    def requests(rate):
        out = []
        for q in WL.serve_requests(n=64, seed=0, arrival_seed=1, rate=rate, steps=steps):
            bx, wg, ph = WL.clap_fling_case(nx=q["nx"], ny=q["ny"], nz=q["nz"], chord=q["chord"],
                                            re=q["re"], j=q["j"], f=q["f"])
            gb, gw = complete_case(bx, wg, ph)

            def u0(q=q, ui=gb["u_in"][0]):
                u = WL.velocity_noise((q["nz"], q["ny"], q["nx"]), 1000 + q["id"])
                u[0] += ui
                return u

            out.append(SweepRequest(rid=q["id"], box=gb, wings=gw, steps=q["steps"],
                                    arrival=q["arrival"], u0=u0, storage=storage))
        return out

    res = {}
    srv = SweepServer(hbm_budget=budget_bytes, chunk=50)
    burst = summarize(srv.run(requests(None)))
    torch.cuda.synchronize()
    burst["max_batch"] = max(srv.batch_sizes)
    burst["peak_bytes"] = srv.peak_bytes
    res["burst"] = burst
    cap = burst["completed"] / burst["span_s"]
    srv = SweepServer(hbm_budget=budget_bytes, chunk=50)
    pois = summarize(srv.run(requests(0.8 * cap)))
    torch.cuda.synchronize()
    pois["rate_per_s"] = 0.8 * cap
    pois["max_batch"] = max(srv.batch_sizes)
    pois["peak_bytes"] = srv.peak_bytes
    res["poisson"] = pois
    return res


def timed_solve(wname, storage, steps, warmup, timing_every):
    """One solve of workload `wname`: `warmup` untimed steps, then `steps`
    timed whole steps bracketed by device synchronisation, with the kernels
    of one step in `timing_every` bracketed by HIP events on the solver's
    stream.  Returns the workload's name, box, foils, physics, initial
    fields and the figures of the timed region."""
    import torch

    from paper_2102_01305_amd.solver import Solver, complete_case

    name, bx, wg, ph = workload(wname)
    if ph["kind"] in ("taylor_green", "lattice"):
        gb, gw = bx, wg
        u0, rho0 = ph["u0"], ph["rho0"]
    else:
        gb, gw = complete_case(bx, wg, ph)
        u0, rho0 = initial_velocity(bx, ph, gb["u_in"][0]), None
    print(f"[bench] {name} storage={storage} tau={gb['tau']:.4f} steps={steps} "
          f"warmup={warmup}", file=sys.stderr, flush=True)
    s = Solver(gb, gw, storage=storage, history_steps=max(steps + warmup, 16))
    s.init_fields(rho=rho0, u=u0)
    N = bx["nx"] * bx["ny"] * bx["nz"]

    s.step(warmup)
    torch.cuda.synchronize()
    s.enable_timing(timing_every)
    s.read_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = s.read_timing()
    s.enable_timing(0)
    # sanity: the solve is still finite
    if gw:
        f = s.forces(s.step_count - 1, 1)
        if not np.all(np.isfinite(f)):
            raise SystemExit("non-finite forces after the timed run")
    else:
        if not np.isfinite(s.mass()[1]):
            raise SystemExit("non-finite mass after the timed run")
    s.close()
    del s
    torch.cuda.empty_cache()

    mlups = N * steps / dt / 1e6
    bpc = 2 * 19 * (4 if storage == "fp32" else 2)
    nl = tim["collide_launches"]
    k6_ms = tim["collide_ms"] / nl if nl else float("nan")
    cells_per_launch = tim["collide_cells"] / nl if nl else float("nan")
    achieved = bpc * cells_per_launch / (k6_ms * 1e-3) / 1e9 if nl else float("nan")
    fig = dict(N=N, dt=dt, mlups=mlups, bpc=bpc, k6_ms=k6_ms, cells_per_launch=cells_per_launch,
               achieved=achieved, launches=nl, marker_ms=tim["marker_ms"] / max(nl, 1))
    return name, bx, wg, ph, u0, rho0, fig


# The storage formats and the largest workload, measured beside the headline
# line of the default run: (workload, storage, steps, warmup).
VARIANTS = (("cf", "fp16", 320, 64), ("cf", "bf16", 320, 64), ("large", "fp32", 64, 64),
            ("large", "fp16", 64, 64), ("tgv", "fp16", 200, 20))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cf")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--timing-every", type=int, default=8,
                    help="bracket the kernels of one step in this many with HIP events")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served sweep")
    ap.add_argument("--serve-budget-gib", type=float, default=4.0,
                    help="HBM budget of the served sweep (admission limit)")
    ap.add_argument("--serve-steps", type=int, default=1000)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other storages and the 512x384x384 solve")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver "
              "has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    name, bx, wg, ph, u0, rho0, fig = timed_solve(args.workload, args.storage, args.steps, args.warmup,
                                                  args.timing_every)
    N, dt, mlups, bpc = fig["N"], fig["dt"], fig["mlups"], fig["bpc"]
    k6_ms, cells_per_launch, achieved = fig["k6_ms"], fig["cells_per_launch"], fig["achieved"]
    traffic = measured_traffic(name, args.storage)
    copy_gbs = copy_bandwidth()
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "cells": N, "storage": args.storage,
                   "re": ph.get("re"), "j": ph.get("j"), "f": ph.get("f"),
                   "wings": len(wg)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_collide", "kernel_ms": round(k6_ms, 5),
                     "bytes_per_cell": bpc, "cells_per_launch": cells_per_launch,
                     "timed_launches": fig["launches"],
                     "marker_ms_per_step": round(fig["marker_ms"], 5),
                     "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "hbm_frac_whole_step": round(mlups * 1e6 * bpc / (HBM_PEAK_GBS * 1e9), 4),
    }
    if not args.no_variants and args.workload == "cf" and args.storage == "fp32":
        # the same measurement for the 16-bit storages and the largest
        # single solve, so one run records every headline configuration
        var = []
        for wv, sv_, kv, wu in VARIANTS:
            vn, _, _, _, _, _, vf = timed_solve(wv, sv_, kv, wu, args.timing_every)
            var.append({"workload": vn, "storage": sv_, "steps": kv, "value": round(vf["mlups"], 1),
                        "ms_per_step": round(vf["dt"] / kv * 1e3, 5),
                        "kernel_ms": round(vf["k6_ms"], 5), "achieved": round(vf["achieved"], 1),
                        "frac": round(vf["achieved"] / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(vn, sv_),
                        "marker_ms_per_step": round(vf["marker_ms"], 5)})
        out["variants"] = var
    if not args.no_serve:
        serving = []
        for sto in ("fp32", "fp16"):
            print(f"[bench] served sweep: 64 requests, {sto}", file=sys.stderr, flush=True)
            sv = serve_bench(int(args.serve_budget_gib * 2**30), args.serve_steps, sto)
            serving.append({
                "requests": 64, "steps_per_request": args.serve_steps,
                "hbm_budget_gib": args.serve_budget_gib, "storage": sto,
                "burst": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in sv["burst"].items()},
                "poisson": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in sv["poisson"].items()},
            })
        out["serving"] = serving
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(name, bx, wg, ph, u0, args.cpu_steps, rho0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
