"""Benchmark of the MI355X QMC step: walker-steps/s on one GPU at n=20.

Workload (default): noisy GHZ preparation on n=20 qubits with non-Markovian dephasing
0.02 cos(0.5 t) and damping 0.002, dt=0.005, 8 replicas x 1e7 walkers, the whole 3000-step
trajectory.  A step is one Euler step of the population dynamics for all replicas (per-step
coefficient table, spawn, child sort, merge with death and annihilation).  Synthetic inputs;
the initial state is resident on the GPU before timing starts.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(kind, st0, st1):
    """Bytes the method must move for one kernel class between two counter snapshots:
    spawn reads each parent record (16 B) and writes each child record (16 B); merge reads
    parents and children and writes the annihilated store (16 B each); the child sort moves
    every child record once in and once out (32 B)."""
    keys = st1["key_steps"] - st0["key_steps"]
    ch = st1["child_steps"] - st0["child_steps"]
    out = st1["out_steps"] - st0["out_steps"]
    if kind == "spawn":
        return 16 * (keys + ch)
    if kind == "merge":
        return 16 * (keys + ch + out)
    return 32 * ch


def cpu_baseline(w, budget_s=20.0):
    """The CPU oracle, untuned, on the host cores over the first steps of the same workload
    (about budget_s seconds of work); reports walker-steps/s."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    o = oracle.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                      w.init_im)
    t0 = time.perf_counter()
    done, used = 0, 1
    chunk = 50
    while done < w.nsteps and time.perf_counter() - t0 < budget_s:
        stop = min(done + chunk, w.nsteps)
        used = o.step(w.s[done:stop], w.gamma[done:stop], threads=threads)
        done = stop
    dt = time.perf_counter() - t0
    c = o.counters()
    return {"value": c["walker_steps"] / dt, "unit": "walker-steps/s", "cores": used,
            "kind": "oracle",
            "sample": f"steps 0..{done} of {w.nsteps} of {w.name} (all {w.n_replicas} replicas), "
                      f"{dt:.1f} s, OpenMP across replicas",
            "key_steps_per_s": c["key_steps"] / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the whole trajectory of the workload)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ghz20_nm", choices=["ghz20_nm", "dd12", "ghz4"])
    ap.add_argument("--roofline-kernel", default="merge", choices=["spawn", "sort", "merge"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(replicas and key-space shards would each map to one GPU).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2502_18929_amd import binding, workloads as W

    w = W.CONFIGS[args.workload]()
    K = w.nsteps if args.steps is None else min(args.steps, w.nsteps)
    Wm = min(args.warmup, w.nsteps)
    caps = {"ghz20_nm": (1 << 17, 1 << 19), "dd12": (1 << 22, 1 << 19), "ghz4": (256, 4096)}
    store_cap, spawn_cap = caps[args.workload]
    torch.cuda.set_device(0)
    g = binding.QMC.from_workload(w, store_capacity=store_cap, spawn_capacity=spawn_cap)
    init = [g.export(r) for r in range(w.n_replicas)]

    # warmup: W steps from the initial state, then restore the initial state (untimed)
    g.run_workload(w, 0, Wm)
    for r in range(w.n_replicas):
        g.import_(r, *init[r], step=0)
    torch.cuda.synchronize()

    st0 = g.counters()
    g.profile(args.roofline_kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run_workload(w, 0, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = g.counters()
    prof_ms, prof_n = g.profile_read()
    g.profile(None)

    elapsed = t1 - t0
    walker_steps = st1["walker_steps"] - st0["walker_steps"]
    key_steps = st1["key_steps"] - st0["key_steps"]
    value = walker_steps / elapsed
    abytes = algorithmic_bytes(args.roofline_kernel, st0, st1)
    achieved = (abytes / prof_n) / (prof_ms / prof_n * 1e-3) / 1e9 if prof_n and prof_ms > 0 else 0.0
    obs = g.observe(pauli=[(x, z) for _, x, z, _ in w.pauli_obs], psi=w.psi)
    nd0 = float(w.walker_target)
    agg_fid = float(obs["fidelity"][:, 0].mean())
    res = {
        "metric": "walker-steps/sec on 1 GPU at n=20; wall time to fixed error bar vs exact",
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": elapsed * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: n={w.n}, {w.n_replicas} replicas x {w.walker_target:g} "
                        f"walkers, dt={w.dt}, {w.nsteps} steps",
            "n_qubits": w.n, "replicas": w.n_replicas, "walker_target": w.walker_target,
            "dt": w.dt, "steps_timed": K, "parallelism": "1 GPU, replicas batched in one store",
        },
        "key_steps_per_s": key_steps / elapsed,
        "roofline": {
            "bound": "hbm", "kernel": args.roofline_kernel,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "avg_launch_ms": prof_ms / prof_n if prof_n else None,
            "launches": prof_n, "algorithmic_bytes_per_launch": abytes / prof_n if prof_n else None,
        },
        "final": {"n_occ_total": st1["n_occ"], "fidelity_mean": agg_fid,
                  "trace_mean": float(obs["trace"].mean())},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w)
    g.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
