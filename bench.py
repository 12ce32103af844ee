"""Benchmark of the MI355X QMC step: walker-steps/s on one GPU at n=20.

Workload (default): noisy GHZ preparation on n=20 qubits with non-Markovian dephasing
0.02 cos(0.5 t) and damping 0.002, dt=0.005, 8 replicas x 1e7 walkers, the whole 3000-step
trajectory.  A step is one Euler step of the population dynamics for all replicas (per-step
coefficient table, death/cloning, spawn, annihilation by key).  Synthetic inputs; the initial
state is resident on the GPU before timing starts.

Prints one JSON line.  --gpus above 1 is refused: the step runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {"fused": "k_persist", "small": "k_small", "sort": "k_onesweep",
                "merge": "k_merge", "step": "streamed_step"}
# the dominant kernel of each workload on the automatic path (with the initiator approximation
# the dd12 store stays small enough for the fused kernel throughout); "fused" stands for the two
# whole-step kernels, timed together, of which the one that ran longer is reported; "step" is
# the whole streamed step (draws, record sort and merge class of every step, timed per chunk of
# steps), reported with the merge class beside it
DOMINANT = {"ghz20_nm": "fused", "dd12": "step", "ghz4": "fused", "batch64": "step"}
DOMINANT_INITIATOR = {"ghz20_nm": "fused", "dd12": "fused", "ghz4": "fused", "batch64": "fused"}
# every source whose change can alter a kernel class's launches or traffic (the host sets the
# launch configuration), so committed counter numbers of a class are dropped as soon as one of
# them changes; which steps a class covered is checked apart (steps per launch)
_CSRC = "paper_2502_18929_amd/csrc/"
_SHARED = [_CSRC + "qmc_device.hpp", _CSRC + "qmc_host.cpp"]
_STREAMED = [_CSRC + "qmc_kernels.hip", _CSRC + "qmc_kernels.h"] + _SHARED
KERNEL_SOURCES = {
    "fused": [_CSRC + "qmc_persist.hip", _CSRC + "qmc_persist.h"] + _SHARED,
    "small": [_CSRC + "qmc_small.hip", _CSRC + "qmc_small.h", _CSRC + "qmc_persist.h"] + _SHARED,
    "step": _STREAMED, "merge": _STREAMED, "sort": _STREAMED,
}


def step_bytes(cov):
    """Algorithmic bytes of whole steps (counter sums `cov` over those steps; 16 B per record:
    u64 key, i32 re, i32 im): read every parent to spawn (16 N_occ), write its diagonal
    (death/cloning) update back (8 N_occ), write and read every off-diagonal child
    (2 x 16 N_sp), read every parent again to annihilate (16 N_occ) and write every surviving key
    (16 N_occ'): 16 (2.5 N_occ + 2 N_sp + N_occ')."""
    return 16 * (2.5 * cov["key_steps"] + 2 * cov["spawn_steps"] + cov["out_steps"])


def algorithmic_bytes(kind, cov):
    """Algorithmic bytes of the steps a kernel class ran.
    fused, small, step: whole steps, so all of step_bytes;
    merge: its annihilation share alone, parents and children read and the store written,
      16 (N_occ + N_sp + N_occ') (the draws of the next step, which it also makes, are left out:
      a lower bound);
    sort: every child read and written once, 32 N_sp."""
    keys, sp, out = cov["key_steps"], cov["spawn_steps"], cov["out_steps"]
    if kind in ("fused", "small", "step"):
        return step_bytes(cov)
    if kind == "merge":
        return 16 * (keys + sp + out)
    return 32 * sp


ERROR_BAR = 0.01  # target half-width of the 95 % confidence interval of the final estimators


def error_bar(obs, w, elapsed, seed=0, boot=2000):
    """95 % bootstrap confidence interval over the replicas (the paper's error bars, End Matter on
    simulation methodology; percentile interval of the mean of resampled replicas) of the final
    fidelity and of every Pauli observable of the workload, and the wall time to the error bar
    ERROR_BAR: the measured run when its widest interval is within it, else the run scaled by
    the replicas the target needs, (h / ERROR_BAR)^2 times as many (replicas are batched in one
    store, so the time grows with them)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    series = {"fidelity": obs["fidelity"][:, 0]}
    for i, (label, _, _, ph) in enumerate(w.pauli_obs):
        v = obs["pauli_val"][:, i, 0] + 1j * obs["pauli_val"][:, i, 1]
        series[label] = (complex(ph) * v).real
    R = len(series["fidelity"])
    if R < 2:
        return None
    idx = rng.integers(0, R, size=(boot, R))
    half = {}
    for k, v in series.items():
        lo, hi = np.percentile(v[idx].mean(axis=1), [2.5, 97.5])
        half[k] = float(hi - lo) / 2
    hmax = max(half.values())
    reached = hmax <= ERROR_BAR
    return {"target_ci95_halfwidth": ERROR_BAR, "replicas": R,
            "ci95_halfwidth_fidelity": half["fidelity"], "ci95_halfwidth_max": hmax,
            "widest": max(half, key=half.get), "reached": reached,
            "wall_s": elapsed if reached else elapsed * (hmax / ERROR_BAR) ** 2,
            "basis": "measured run" if reached else "extrapolated: replicas x (h / target)^2"}


def sources_digest(kind):
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(kind, workload, steps_per_launch):
    """HBM bytes per launch of the kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None when there is no
    summary for this kernel and workload, when its launches covered another number of steps than
    the ones timed here, or when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{KERNEL_NAMES[kind]}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"sources_digest:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    c = re.search(r"steps_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not b or not c or m.group(1) != sources_digest(kind):
        return None
    if steps_per_launch is None or abs(float(c.group(1)) - steps_per_launch) > 1e-9:
        return None
    return float(b.group(1))


def host_description():
    """Host cores and CPU model of the machine the CPU baseline runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(w, K, integrator="euler", init_min=0, budget_s=10.0, proposal=None):
    """The CPU oracle, untuned, on the host cores over the same steps [0, K) that the GPU timed,
    from the same initial state: the window is run again from the start until about budget_s
    seconds of work are done, or cut at budget_s when one pass takes longer.  Reports
    walker-steps/s over everything it ran.  proposal = (kind, samples, mlp) or None (the comb)."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    ws = ks = 0
    passes, done, used = 0, 0, 1
    chunk = 50
    while time.perf_counter() - t0 < budget_s:
        o = oracle.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                          w.init_im, integrator=integrator)
        o.set_initiator(init_min)
        if proposal:
            o.set_proposal(*proposal)
        done = 0
        for a, b, pulses in w.segments():
            if a >= K or time.perf_counter() - t0 >= budget_s:
                break
            for (px, pz) in pulses:
                o.pulse(px, pz)
            for lo in range(a, min(b, K), chunk):
                if time.perf_counter() - t0 >= budget_s:
                    break
                hi = min(lo + chunk, b, K)
                used = o.step(w.s[lo:hi], w.gamma[lo:hi], threads=threads)
                done = hi
        c = o.counters()
        ws += c["walker_steps"]
        ks += c["key_steps"]
        o.close()
        if done < K:
            break
        passes += 1
    dt = time.perf_counter() - t0
    partial = done if done < K else 0
    if partial == 0:
        what = f"{passes} pass(es) over steps 0..{K}"
    elif passes == 0:
        what = f"steps 0..{partial} of the timed window 0..{K}"
    else:
        what = f"{passes} pass(es) over steps 0..{K} and steps 0..{partial} of one more"
    return {"value": ws / dt, "unit": "walker-steps/s", "cores": used, "kind": "oracle",
            "sample": f"{what} of {w.name} (all {w.n_replicas} replicas, the GPU's timed "
                      f"window), {dt:.1f} s, OpenMP across replicas",
            "key_steps_per_s": ks / dt, "host": host_description()}


def whole_step_class(g, kind):
    """The timed class's totals.  The two whole-step kernels (fused persistent, LDS-resident) are
    timed together: the one that ran longer is the one reported, the other's time and launches
    are returned beside it.  The whole streamed step comes with the merge class's own roofline
    (its annihilation bytes alone) beside it."""
    if kind == "step":
        ms, n, cov = g.profile_read("step")
        mms, mn, mcov = g.profile_read("merge")
        m = roofline("merge", None, mms, mn, mcov)
        other = {"merge_class": {k: m[k] for k in ("achieved", "frac", "avg_launch_ms",
                                                   "launches", "algorithmic_bytes_per_launch")}}
        return kind, ms, n, cov, other
    if kind not in ("fused", "small"):
        ms, n, cov = g.profile_read()
        return kind, ms, n, cov, None
    got = {k: g.profile_read(k) for k in ("fused", "small")}
    top = max(got, key=lambda k: got[k][0])
    low = "small" if top == "fused" else "fused"
    ms, n, cov = got[top]
    other = {"kernel": KERNEL_NAMES[low], "ms": got[low][0], "launches": got[low][1],
             "steps_covered": got[low][2]["steps"]}
    return top, ms, n, cov, other


def roofline(kind, workload, prof_ms, prof_n, cov):
    """The roofline object of the timed kernel class: algorithmic bytes per launch over the
    average launch duration (HIP events on the context stream around exactly those launches),
    against the HBM peak; the whole-step bytes of the same steps beside it."""
    abytes = algorithmic_bytes(kind, cov)
    per_launch = abytes / prof_n if prof_n else None
    avg_ms = prof_ms / prof_n if prof_n else None
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if prof_n and prof_ms > 0 else 0.0
    spl = cov["steps"] / prof_n if prof_n else None
    # the per-step latency of the class (the honest measure where a step's bytes take far less
    # HBM time than its chain of dependent operations)
    us_step = avg_ms * 1e3 / spl if prof_n and spl else None
    return {"bound": "hbm", "kernel": KERNEL_NAMES[kind], "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(kind, workload, spl), "avg_launch_ms": avg_ms,
            "kernel_us_per_step": us_step,
            "launches": prof_n, "steps_covered": cov["steps"], "steps_per_launch": spl,
            "algorithmic_bytes_per_launch": per_launch,
            "step_bytes_per_launch": step_bytes(cov) / prof_n if prof_n else None,
            "counts": {k: cov[k] for k in ("key_steps", "spawn_steps", "child_steps",
                                           "out_steps")}}


EXACT_PATH = os.path.join(ROOT, "tests", "golden", "ghz4_exact.json")


def vs_exact(obs, w, integrator):
    """Replica means of the final estimators against the dense solutions of the same model
    (stored by tests/golden/make_exact.py): the dense map of the integrator used, which is the
    exact expectation of the stochastic step (z-score over the replicas), and the exact
    propagation (the integrator's time-step bias beside the statistical error)."""
    import numpy as np
    if not os.path.exists(EXACT_PATH):
        return None
    ref = json.load(open(EXACT_PATH))
    if ref.get("workload") != w.name or ref.get("nsteps") != w.nsteps:
        return None
    series = {"fidelity": obs["fidelity"][:, 0], "trace": obs["trace"]}
    for i, (label, _, _, ph) in enumerate(w.pauli_obs):
        v = obs["pauli_val"][:, i, 0] + 1j * obs["pauli_val"][:, i, 1]
        series[label] = (complex(ph) * v).real
    mp = "ab2_map" if integrator == "ab2" else "euler_map"
    out = {}
    for k, v in series.items():
        mean = float(np.mean(v))
        se = float(np.std(v, ddof=1) / np.sqrt(len(v))) if len(v) > 1 else float("nan")
        m, ex = ref[mp][k], ref["expm"][k]
        out[k] = {"mean": mean, "se": se, mp: m, "expm": ex,
                  "z_vs_map": (mean - m) / se if se > 0 else None,
                  "dev_vs_expm": mean - ex, "map_bias_vs_expm": m - ex}
    zs = [abs(o["z_vs_map"]) for o in out.values() if o["z_vs_map"] is not None]
    return {"reference": mp, "max_abs_z_vs_map": max(zs) if zs else None,
            "max_abs_dev_vs_expm": max(abs(o["dev_vs_expm"]) for o in out.values()),
            "observables": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the whole trajectory of the workload)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ghz20_nm",
                    choices=["ghz20_nm", "dd12", "ghz4", "batch64"])
    ap.add_argument("--path", default="auto", choices=["auto", "fused", "streamed", "small"])
    ap.add_argument("--integrator", default="euler", choices=["euler", "ab2"],
                    help="time integrator (End Matter on simulation methodology)")
    ap.add_argument("--roofline-kernel", default=None, choices=list(KERNEL_NAMES),
                    help="kernel class timed for the roofline (default: the workload's "
                         "dominant kernel)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB before the timed region (the "
                         "known-size kernel that calibrates HBM counter runs)")
    ap.add_argument("--initiator-xi", default=None,
                    help="initiator approximation with threshold xi * N^diag (End Matter on "
                         "simulation methodology; the paper uses 0.001); default: the plain step")
    ap.add_argument("--proposal", default="comb", choices=["comb", "uniform", "heatbath", "mlp"],
                    help="spawn proposal (End Matter spawn step, importance weighted); mlp is "
                         "trained first on statistics of an untimed plain run")
    ap.add_argument("--proposal-samples", type=int, default=4,
                    help="channel draws per parent under a proposal (a power of two)")
    ap.add_argument("--pulse-width", type=float, default=None,
                    help="dd12 with square pulses of this width instead of ideal instantaneous "
                         "ones")
    ap.add_argument("--pulse-substeps", type=int, default=10,
                    help="steps per dt inside finite pulse windows")
    ap.add_argument("--sequential-steps", type=int, default=0,
                    help="batch64: also time its first this many steps circuit by circuit, one "
                         "context each, against the batched step")
    ap.add_argument("--compare-proposals", action="store_true",
                    help="ghz20_nm: the learned proposal (the deeper int8 network, trained first on "
                         "the spawn events of a plain run) against uniform, heat-bath and the "
                         "comb: sign angle and the <Z0>(t) error bar at equal wall time")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--graphs", action="store_true",
                    help="capture each chunk of streamed steps into a HIP graph and replay it")
    ap.add_argument("--progress", type=int, default=0,
                    help="print a line to stderr after every this many timed steps (runs the "
                         "timed region in calls of that many steps; 0: one call)")
    args = ap.parse_args()
    if args.pulse_width is not None and (args.workload != "dd12" or args.integrator != "euler"):
        ap.error("--pulse-width applies to dd12 with the Euler step (AB2 needs a uniform step)")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(replicas and key-space shards would each map to one GPU).", file=sys.stderr)
        sys.exit(2)
    if args.compare_proposals:
        return compare_proposals(args)
    dominant = DOMINANT_INITIATOR if args.initiator_xi else DOMINANT
    kind = args.roofline_kernel or ("step" if args.path == "streamed" or
                                    args.proposal != "comb" else dominant[args.workload])

    import torch
    from paper_2502_18929_amd import binding, workloads as W

    if args.workload == "batch64":
        return main_batch(args, kind)
    w = (W.CONFIGS[args.workload]() if args.pulse_width is None else
         W.config_dd12(pulse_width=args.pulse_width, substeps=args.pulse_substeps))
    K = w.nsteps if args.steps is None else min(args.steps, w.nsteps)
    Wm = min(args.warmup, w.nsteps)
    caps = {"ghz20_nm": (1 << 17, 1 << 19), "dd12": (1 << 24, 1 << 21), "ghz4": (256, 4096)}
    store_cap, spawn_cap = caps[args.workload]
    torch.cuda.set_device(0)
    g = binding.QMC.from_workload(w, store_capacity=store_cap, spawn_capacity=spawn_cap)
    g.set_path(args.path)
    g.use_graphs(args.graphs)
    g.set_integrator(args.integrator)
    init_min = (binding.initiator_threshold(args.initiator_xi, w.walker_target)
                if args.initiator_xi else 0)
    g.set_initiator(init_min)
    init = [g.export(r) for r in range(w.n_replicas)]
    # the tile of the look-back sort that re-sorts the store after an x pulse, autotuned where
    # the streamed path carries the run (the per-step sort has fixed tiles)
    sort_tile = g.tune_sort(0 if (args.path == "streamed" or args.proposal != "comb" or
                                  DOMINANT[args.workload] != "fused") else 16)
    prop, train_corr = None, None
    if args.proposal != "comb":
        mlp = None
        if args.proposal == "mlp":
            # statistics of the method's own plain run (untimed), then back to the initial state
            from paper_2502_18929_amd import proposal as PR
            at = list(range(w.nsteps // 16, w.nsteps, w.nsteps // 16))
            mlp, train_corr = PR.train(g, w, at[-1])
            for r in range(w.n_replicas):
                g.import_(r, *init[r], step=0)
        prop = (args.proposal, args.proposal_samples, mlp)
        g.set_proposal(*prop)

    # warmup: W steps from the initial state under the same instrumentation as the timed steps
    # (the first timed launches of a process otherwise pay the event set-up), then restore the
    # initial state (untimed); the timing totals start again below
    # per-class timing events are not recorded inside captured graphs: with --graphs the chunks
    # run captured and uninstrumented, and the line carries no roofline
    prof = None if args.graphs else kind
    g.profile(prof)
    g.run_workload(w, 0, Wm)
    for r in range(w.n_replicas):
        g.import_(r, *init[r], step=0)
    g.set_integrator(args.integrator)  # forget the warmup's N(s-1): the run starts at step 0
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib << 18  # float32 elements
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        del a, b
    torch.cuda.synchronize()

    st0 = g.counters()
    g.profile(prof)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.progress > 0:
        for a in range(0, K, args.progress):
            g.run_workload(w, a, min(a + args.progress, K))
            print(f"timed steps {a}..{min(a + args.progress, K)}", file=sys.stderr, flush=True)
    else:
        g.run_workload(w, 0, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = g.counters()
    elapsed = t1 - t0
    walker_steps = st1["walker_steps"] - st0["walker_steps"]
    key_steps = st1["key_steps"] - st0["key_steps"]
    value = walker_steps / elapsed
    if prof:
        kind, prof_ms, prof_n, cov, other = whole_step_class(g, kind)
        g.profile(None)
        roof = roofline(kind, w.name, prof_ms, prof_n, cov)
        if other and kind == "step":
            roof.update(other)
        elif other:
            roof["other_whole_step_kernel"] = other
    else:
        roof = None
    obs = g.observe(pauli=[(x, z) for _, x, z, _ in w.pauli_obs], psi=w.psi)
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
            "dt": w.dt, "steps_timed": K, "step_path": args.path, "graphs": args.graphs,
            "notes": w.notes,
            "integrator": args.integrator,
            "initiator": ({"xi": args.initiator_xi, "min_walkers": init_min}
                          if init_min else None),
            "parallelism": "1 GPU, replicas batched in one store",
            "pulse_sort_tile_records_per_thread": sort_tile,
        },
        "key_steps_per_s": key_steps / elapsed,
        "rebalances": st1["rebalances"] - st0["rebalances"],
        "roofline": roof,
        "final": {"n_occ_total": st1["n_occ"], "t": K * w.dt,
                  "fidelity_mean": float(obs["fidelity"][:, 0].mean()),
                  "fidelity_std_replicas": float(obs["fidelity"][:, 0].std(ddof=1)),
                  "trace_mean": float(obs["trace"].mean()),
                  "error_bar": (error_bar(obs, w, elapsed) if K == w.nsteps else None),
                  "error_bar_note": (None if K == w.nsteps else
                                     f"the timed window ends at step {K} of {w.nsteps}: the "
                                     "error bar is taken at the end of the trajectory only")},
    }
    if w.n <= 5 and K == w.nsteps:
        res["vs_exact"] = vs_exact(obs, w, args.integrator)
    if prop:
        res["config"]["proposal"] = {"kind": prop[0], "samples": prop[1],
                                     "mlp_train_corr": train_corr}
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w, K, args.integrator, init_min, proposal=prop)
    g.close()
    print(json.dumps(res), flush=True)


def cpu_baseline_batch(bw, K, budget_s=20.0):
    """The CPU oracle, circuit by circuit (each with its replicas' stream ids), over the steps
    [0, K) the GPU timed, cut at about budget_s seconds; walker-steps/s over all circuits."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    R = bw.n_replicas
    orcs = []
    for c, w in enumerate(bw.circuits):
        o = oracle.Oracle(bw.n, R, bw.seed, bw.dt, w.h, w.lops, w.init_keys, w.init_re,
                          w.init_im)
        o.set_replica_base(c * R)
        orcs.append(o)
    t0 = time.perf_counter()
    done, used = 0, 1
    for a, b, masks in bw.segments():
        if a >= K:
            break
        for lo in range(a, min(b, K), 20):
            if time.perf_counter() - t0 >= budget_s:
                break
            hi = min(lo + 20, b, K)
            if lo == a and masks is not None:
                for c, o in enumerate(orcs):
                    if masks[0][c] or masks[1][c]:
                        o.pulse(int(masks[0][c]), int(masks[1][c]))
            for o, w in zip(orcs, bw.circuits):
                used = max(used, o.step(w.s[lo:hi], w.gamma[lo:hi], threads=threads))
            done = hi
    dt = time.perf_counter() - t0
    ws = sum(o.counters()["walker_steps"] for o in orcs)
    ks = sum(o.counters()["key_steps"] for o in orcs)
    return {"value": ws / dt, "unit": "walker-steps/s", "cores": used, "kind": "oracle",
            "sample": f"steps 0..{done} of the timed window 0..{K} of {bw.name} (all "
                      f"{len(orcs)} circuits x {R} replicas), {dt:.1f} s, OpenMP across each "
                      f"circuit's replicas",
            "key_steps_per_s": ks / dt, "host": host_description()}


def batch_vs_oracle(g, bw, init, K, S=1):
    """Per-circuit check of the batched run at its last step, by the CPU oracle: the context goes
    back to the initial state and runs to step K - S, every circuit's replicas are imported into
    an oracle of that circuit (stream ids c R + r, the state is (store, step) since the draws are
    keyed on the walkers), and both take the last S steps.  A circuit's flag is true when every
    one of its replicas' stores is identical (keys and both counts)."""
    import numpy as np
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    R = bw.n_replicas
    for r in range(g.R):
        g.import_(r, *init[r], step=0)
    g.run_batch_workload(bw, 0, K - S)
    orcs = []
    for c, w in enumerate(bw.circuits):
        o = oracle.Oracle(bw.n, R, bw.seed, bw.dt, w.h, w.lops, w.init_keys, w.init_re,
                          w.init_im)
        o.set_replica_base(c * R)
        for r in range(R):
            o.import_(r, *g.export(c * R + r), step=K - S)
        orcs.append(o)
    t0 = time.perf_counter()
    for a, b, masks in bw.segments():
        if b <= K - S or a >= K:
            continue
        if a >= K - S and masks is not None:
            for c, o in enumerate(orcs):
                if masks[0][c] or masks[1][c]:
                    o.pulse(int(masks[0][c]), int(masks[1][c]))
        lo, hi = max(a, K - S), min(b, K)
        for o, w in zip(orcs, bw.circuits):
            o.step(w.s[lo:hi], w.gamma[lo:hi], threads=threads)
    g.run_batch_workload(bw, K - S, K)
    flags = []
    for c, o in enumerate(orcs):
        ok = True
        for r in range(R):
            x, y = g.export(c * R + r), o.export(r)
            ok = ok and all(np.array_equal(u, v) for u, v in zip(x, y))
        flags.append(bool(ok))
        o.close()
    return {"steps_checked": f"{K - S}..{K}", "circuits": len(flags),
            "bit_exact": flags, "all_bit_exact": all(flags),
            "oracle_s": time.perf_counter() - t0}


def batch_vs_sequential(bw, S, path):
    """The first S steps of the batch twice: batched (all circuits in one context) and circuit by
    circuit (one context each, run one after another), wall times between device
    synchronizations.  The batched step equals each circuit's own step bit for bit (tested), so
    the statistics are the same and the time ratio is what batching gains."""
    import torch
    from paper_2502_18929_amd import binding
    circuits = [(w.h, w.lops, w.init_keys, w.init_re, w.init_im) for w in bw.circuits]
    g = binding.QMC.batch(bw.n, bw.n_replicas, bw.seed, bw.dt, circuits,
                          store_capacity=1 << 18, spawn_capacity=1 << 18)
    g.set_path(path)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run_batch_workload(bw, 0, S)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    g.close()
    t_seq = 0.0
    for w in bw.circuits:
        q = binding.QMC.from_workload(w, store_capacity=1 << 21, spawn_capacity=1 << 21)
        q.set_path(path)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q.run_workload(w, 0, S)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        q.close()
    return {"steps": S, "circuits": len(bw.circuits), "batched_s": t_batch,
            "sequential_s": t_seq, "speedup": t_seq / t_batch}


def main_batch(args, kind):
    """The batched configuration: 64 circuits of uneven size in one context and one step."""
    import torch
    from paper_2502_18929_amd import binding, workloads as W
    bw = W.config_batch64()
    K = bw.nsteps if args.steps is None else min(args.steps, bw.nsteps)
    Wm = min(args.warmup, bw.nsteps)
    torch.cuda.set_device(0)
    circuits = [(w.h, w.lops, w.init_keys, w.init_re, w.init_im) for w in bw.circuits]
    g = binding.QMC.batch(bw.n, bw.n_replicas, bw.seed, bw.dt, circuits,
                          store_capacity=1 << 18, spawn_capacity=1 << 18)
    g.set_path(args.path)
    g.use_graphs(args.graphs)
    init = [g.export(r) for r in range(g.R)]
    sort_tile = g.tune_sort(0)   # the store re-sort after an x pulse (streamed path)
    prof = None if args.graphs else kind  # captured graphs carry no per-class timing events
    g.profile(prof)              # the warmup under the timed steps' instrumentation
    g.run_batch_workload(bw, 0, Wm)
    for r in range(g.R):
        g.import_(r, *init[r], step=0)
    torch.cuda.synchronize()
    st0 = g.counters()
    g.profile(prof)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run_batch_workload(bw, 0, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = g.counters()
    elapsed = t1 - t0
    walker_steps = st1["walker_steps"] - st0["walker_steps"]
    roof = None
    if prof:
        kind, prof_ms, prof_n, cov, other = whole_step_class(g, kind)
        g.profile(None)
        roof = roofline(kind, bw.name, prof_ms, prof_n, cov)
        if other and kind == "step":
            roof.update(other)
        elif other:
            roof["other_whole_step_kernel"] = other
    obs = g.observe()
    res = {
        "metric": "walker-steps/sec on 1 GPU (batched circuits)",
        "value": walker_steps / elapsed, "unit": "walker-steps/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": elapsed * 1e3 / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"{bw.name}: {len(bw.circuits)} circuits, n = "
                               f"{min(w.n for w in bw.circuits)}..{max(w.n for w in bw.circuits)}"
                               f" (DD or GHZ), {bw.n_replicas} replicas each, walker targets "
                               f"1e4..1e6, dt={bw.dt}, {bw.nsteps} steps",
                   "circuits": len(bw.circuits), "replicas": bw.n_replicas, "dt": bw.dt,
                   "steps_timed": K, "step_path": args.path, "graphs": args.graphs,
                   "parallelism": "1 GPU, all circuits and replicas in one store",
                   "pulse_sort_tile_records_per_thread": sort_tile},
        "key_steps_per_s": (st1["key_steps"] - st0["key_steps"]) / elapsed,
        "roofline": roof,
        "final": {"n_occ_total": st1["n_occ"], "trace_mean": float(obs["trace"].mean())},
    }
    if args.sequential_steps > 0:
        res["batched_vs_sequential"] = batch_vs_sequential(bw, min(args.sequential_steps, K),
                                                           args.path)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_batch(bw, K)
        # the CPU leg also checks every circuit against the oracle at the end of the timed window
        res["cpu_baseline"]["per_circuit_vs_oracle"] = batch_vs_oracle(g, bw, init, K)
    g.close()
    print(json.dumps(res), flush=True)


def _ci95(v, boot=2000, seed=0):
    """Half-width of the 95 % bootstrap percentile interval of the mean of v over replicas."""
    import numpy as np
    rng = np.random.default_rng(seed)
    v = np.asarray(v, dtype=np.float64)
    if len(v) < 2:
        return float("nan")
    m = v[rng.integers(0, len(v), size=(boot, len(v)))].mean(axis=1)
    lo, hi = np.percentile(m, [2.5, 97.5])
    return float(hi - lo) / 2


def compare_proposals(args):
    """The learned proposal against uniform, heat-bath and the plain comb on ghz20_nm (8 replicas,
    3000 steps, K draws per parent): the deeper int8 network is trained first (untimed) on the
    off-diagonal spawn events of a plain run; then each kind runs the whole trajectory from the
    initial state, and at every 250 steps the replicas' sign angle theta = arg N^diag (End Matter
    on sign-problem suppression), Re N^diag and <Z0> are read.  The <Z0>(t) error bar is the 95 %
    bootstrap half-width over the replicas; at equal wall time it is scaled by
    sqrt(time / time of the comb) (replicas cost time linearly, the error bar falls as their
    square root)."""
    import numpy as np
    import torch
    from paper_2502_18929_amd import binding, proposal as PR, workloads as W
    torch.cuda.set_device(0)
    w = W.config_ghz20_nm()
    store, spawn = 1 << 17, 1 << 19
    K = args.proposal_samples
    t0 = time.perf_counter()
    tr = binding.QMC.from_workload(w, store_capacity=store, spawn_capacity=spawn)
    net, info = PR.train_deep(tr, w)
    tr.close()
    info["train_s"] = time.perf_counter() - t0
    z0 = [i for i, (lab, _, _, _) in enumerate(w.pauli_obs) if lab == "Z0"][0]
    pauli = [(x, z) for _, x, z, _ in w.pauli_obs]
    ph = complex(w.pauli_obs[z0][3])
    every = 250
    out = {}
    for kind in ("comb", "uniform", "heatbath", "learned"):
        g = binding.QMC.from_workload(w, store_capacity=store, spawn_capacity=spawn)
        if kind == "learned":
            g.set_proposal_deep(K, net)
        elif kind != "comb":
            g.set_proposal(kind, K)
        torch.cuda.synchronize()
        el = 0.0
        rows = []
        for a in range(0, w.nsteps, every):
            b = min(a + every, w.nsteps)
            t1 = time.perf_counter()
            g.run_workload(w, a, b)
            torch.cuda.synchronize()
            el += time.perf_counter() - t1
            obs = g.observe(pauli=pauli, psi=w.psi)
            zv = (ph * (obs["pauli_val"][:, z0, 0] + 1j * obs["pauli_val"][:, z0, 1])).real
            nd = obs["ndiag"][:, 0].astype(np.float64)
            rows.append({"step": b, "theta_abs_mean": float(np.abs(obs["theta"]).mean()),
                         "theta_abs_max": float(np.abs(obs["theta"]).max()),
                         "re_ndiag_rel": float(nd.mean() / w.walker_target),
                         "z0_mean": float(zv.mean()), "z0_ci95": _ci95(zv),
                         "fidelity_mean": float(obs["fidelity"][:, 0].mean())})
        out[kind] = {"wall_s": el, "ms_per_step": el * 1e3 / w.nsteps, "series": rows}
        g.close()
    base = out["comb"]["wall_s"]
    for kind, o in out.items():
        scale = np.sqrt(o["wall_s"] / base)
        cis = np.array([r["z0_ci95"] for r in o["series"]])
        o["z0_ci95_at_tf"] = float(cis[-1])
        o["z0_ci95_equal_time_at_tf"] = float(cis[-1] * scale)
        o["z0_ci95_equal_time_max"] = float(np.nanmax(cis) * scale)
        o["theta_abs_max"] = max(r["theta_abs_max"] for r in o["series"])
    res = {"metric": "learned spawn proposal against uniform, heat-bath and the comb at equal "
                     "wall time (sign angle, <Z0>(t) error bar)",
           "workload": f"{w.name}: n={w.n}, {w.n_replicas} replicas x {w.walker_target:g} walkers, "
                       f"dt={w.dt}, {w.nsteps} steps",
           "samples_per_parent": K, "training": info, "kinds": out, "dtype": "int64",
           "data": "synthetic"}
    print(json.dumps(res), flush=True)


def release_device():
    """Everything this process holds on the device is given back before the interpreter exits:
    contexts are closed by then, so only torch's cached blocks remain."""
    import gc
    import torch
    gc.collect()
    if torch.cuda.is_available():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
    release_device()
