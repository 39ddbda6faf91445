"""Write the FP64 oracle's reference for clap & fling at the benchmark size.

Workload: two elliptic foils (chord 20, aspect 5) in a 256x192x192 box,
Re = 100, J = 0.01, f = 0.25 (Sec. 3.3-3.4), initial velocity U_inf plus
seeded noise (seed 0), run over one full flapping period (ceil(T) steps, two
clap and fling events, Eq. 23 read as |sin|).  Calls only the oracle
(`oracle.sim.Sim` with its C lattice) and the input generators in
`workloads`; nothing here comes from the GPU library.

Output (npz, float64):
  history     [steps][2][8]  Fx, Fy, Fz, Mz, CL, CT, CD, CM of each foil
  sample_idx  [n]            flat cell indices (x fastest) of the u sample
  u_sample    [3][n]         u* of the state after `sample_step` steps
  rho_sample  [n]            rho of that state
  sample_step                200
  The sample is 10,000 cells drawn uniformly over the box and 10,000 drawn
  from the delta-kernel support nodes of both foils' markers (PCG64 seed 2102).

    python tests/golden/make_clap_fling_period.py [--threads 6] [--checkpoint-dir DIR]

About 75 minutes on 6 host cores.  With --checkpoint-dir the state is saved
every 200 steps there and a rerun resumes from the last save.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "clap_fling_256x192x192_period.npz")
CASE = dict(nx=256, ny=192, nz=192, chord=20.0, re=100.0, j=0.01, f=0.25)
NOISE_SEED = 0
SAMPLE_STEP = 200
SAMPLE_SEED = 2102
N_UNIFORM = 10000
N_SUPPORT = 10000


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--checkpoint-dir", default=None)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    os.environ["OMP_NUM_THREADS"] = str(args.threads)

    import numpy as np

    import workloads as WL
    from oracle import params
    from oracle.sim import Sim

    bx, wg, ph = WL.clap_fling_case(**CASE)
    ob, ow = params.complete_case(bx, wg, ph)
    steps = int(math.ceil(ow[0]["period_steps"]))
    u0 = WL.velocity_noise((bx["nz"], bx["ny"], bx["nx"]), NOISE_SEED)
    u0[0] += ob["u_in"][0]
    sim = Sim(ob, ow, u0=u0, lattice="c")
    N = sim.N
    sample = None
    ck = args.checkpoint_dir
    if ck:
        os.makedirs(ck, exist_ok=True)
        meta_p = os.path.join(ck, "meta.json")
        if os.path.exists(meta_p):
            with open(meta_p) as fh:
                meta = json.load(fh)
            sim.S = np.load(os.path.join(ck, "S.npy"))
            sim.n = meta["n"]
            sim.history = list(np.load(os.path.join(ck, "history.npy")))
            if os.path.exists(os.path.join(ck, "sample.npz")):
                z = np.load(os.path.join(ck, "sample.npz"))
                sample = (z["idx"], z["u"], z["rho"])
            print(f"[golden] resumed at step {sim.n}", flush=True)
    t0 = time.time()
    while sim.n < steps:
        sim.step()
        if sim.n == SAMPLE_STEP:
            rho, u = sim.fields()
            rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
            uni = rng.choice(N, size=N_UNIFORM, replace=False)
            sup = np.unique(sim.last["nodes"].ravel())
            sup = np.setdiff1d(sup, uni)
            near = rng.choice(sup, size=N_SUPPORT, replace=False)
            idx = np.sort(np.concatenate([uni, near])).astype(np.int64)
            sample = (idx, u.reshape(3, -1)[:, idx].copy(), rho.reshape(-1)[idx].copy())
            if ck:
                np.savez(os.path.join(ck, "sample.npz"), idx=sample[0], u=sample[1], rho=sample[2])
        if sim.n % 50 == 0:
            h = np.array(sim.history[-1])
            print(f"[golden] step {sim.n}/{steps}  {time.time() - t0:.0f} s  CL {h[0, 4]:+.4e} {h[1, 4]:+.4e}",
                  flush=True)
        if ck and sim.n % 200 == 0:
            np.save(os.path.join(ck, "S.npy"), sim.S)
            np.save(os.path.join(ck, "history.npy"), np.array(sim.history))
            with open(os.path.join(ck, "meta.json"), "w") as fh:
                json.dump({"n": sim.n}, fh)
    hist = np.array(sim.history)
    meta = dict(case=CASE, noise_seed=NOISE_SEED, steps=steps, period_steps=ow[0]["period_steps"],
                tau=ob["tau"], u_in=ob["u_in"][0], u_ref=ob["u_ref"], sample_seed=SAMPLE_SEED,
                generator="tests/golden/make_clap_fling_period.py (oracle.sim.Sim, lattice='c')")
    np.savez_compressed(args.out, history=hist, sample_idx=sample[0], u_sample=sample[1],
                        rho_sample=sample[2], sample_step=np.int64(SAMPLE_STEP),
                        meta=np.array(json.dumps(meta)))
    print(f"[golden] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
