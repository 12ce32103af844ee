"""GPU parity at the sizes the oracle cannot follow from step 0: GPU states imported into the oracle.

The Philox streams are keyed on (walker key, step, replica), so a store and its step number are
the complete state of a replica (End Matter on spawn and annihilation: each step depends on N(t)
alone).  At a few steps of the full-size runs -- dd12 up to 121M keys, all 64 circuits of the
batched configuration -- the GPU stores are exported, imported into the oracle at the same step,
and both sides then take the next steps on their own: every replica must stay identical, bit for
bit.  The estimator numerators of eq. (3) (occupied keys, N^tot, N^diag, Pauli sums, fidelity
lookups, anti-Hermiticity) are compared on the same imported states, and the step counters the
benchmark's algorithmic bytes come from are compared with the oracle's on whole trajectories.
"""
import sys
import time

import numpy as np
import pytest

from paper_2502_18929_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_18929_amd import binding
    binding.lib()
    return binding


def _same_store(a, b, where):
    ka, aa, ba = a
    kb, ab, bb = b
    if not (np.array_equal(ka, kb) and np.array_equal(aa, ab) and np.array_equal(ba, bb)):
        n = min(len(ka), len(kb))
        bad = np.nonzero((ka[:n] != kb[:n]) | (aa[:n] != ab[:n]) | (ba[:n] != bb[:n]))[0]
        first = int(bad[0]) if len(bad) else n
        raise AssertionError(f"{where}: sizes gpu {len(ka)} oracle {len(kb)}, first difference "
                             f"at {first}")


def _check_observe(g, orcs, w, pauli, where):
    """GPU estimator numerators against the oracle's on the same states: orcs maps each GPU
    segment to (oracle, its replica index)."""
    got = g.observe(pauli=pauli, psi=w.psi, want_eps=True)
    lk = [(v << w.n) | u for u, _ in w.psi for v, _ in w.psi]
    for seg, (o, r) in orcs.items():
        ref = o.observe(r, pauli, lk)
        assert int(got["n_occ"][seg]) == ref["n_occ"], (where, seg)
        assert int(got["n_tot"][seg]) == ref["n_tot"], (where, seg)
        assert tuple(got["ndiag"][seg]) == ref["ndiag_int"], (where, seg)
        assert np.array_equal(got["pauli"][seg], ref["pauli"]), (where, seg)
        assert got["eps2_int"][seg] == ref["eps2"], (where, seg)
        F, idx = 0.0, 0
        for _, au in w.psi:
            for _, av in w.psi:
                F += (np.conj(au) * av * complex(*ref["lookup"][idx])).real
                idx += 1
        assert abs(got["fidelity"][seg, 0] - F / float(w.walker_target)) < 1e-12, (where, seg)


def _extra_paulis(n, count, seed):
    rng = np.random.default_rng(seed)
    m = (1 << n) - 1
    return [(int(rng.integers(0, m + 1)), int(rng.integers(0, m + 1))) for _ in range(count)]


# ---- step counters (the algorithmic bytes of the benchmark) ----------------------------------

@pytest.mark.parametrize("path", ["fused", "streamed"])
@pytest.mark.parametrize("case", ["ghz4", "dd6"])
def test_counters_match_oracle(B, orc, path, case):
    """Over whole trajectories the GPU's running sums of N^tot, occupied parent keys and
    off-diagonal child records equal the oracle's (the death/cloning deltas, which the GPU
    routes as records, are not children)."""
    if case == "ghz4":
        w, store, spawn = W.config_ghz4(), 256, 4096
    else:
        w = W.dd(n=6, n_replicas=4, walker_target=20000, nsteps=500, seed=12)
        store, spawn = 4096, 1 << 16
    g = B.QMC.from_workload(w, store_capacity=store, spawn_capacity=spawn)
    g.set_path(path)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    for a, b, pulses in w.segments():
        for (px, pz) in pulses:
            g.pulse(px, pz)
            o.pulse(px, pz)
        g.step(w.s[a:b], w.gamma[a:b])
        o.step(w.s[a:b], w.gamma[a:b])
    gc, oc = g.counters(), o.counters()
    assert gc["walker_steps"] == oc["walker_steps"]
    assert gc["key_steps"] == oc["key_steps"]
    assert gc["spawn_steps"] == oc["child_steps"]
    assert gc["child_steps"] >= gc["spawn_steps"]


@pytest.mark.timeout(600)
def test_counters_match_oracle_ghz20_nm(B, orc):
    """The same on the benchmarked workload at full size (3000 steps, automatic path: the fused
    kernel re-cuts its key ranges inside its launches and draws those steps' records again)."""
    w = W.config_ghz20_nm()
    g = B.QMC.from_workload(w, store_capacity=1 << 17, spawn_capacity=1 << 19)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    g.step(w.s, w.gamma)
    o.step(w.s, w.gamma, threads=16)
    gc, oc = g.counters(), o.counters()
    _say(f"ghz20_nm counters: gpu {gc}, oracle {oc}")
    assert gc["rebalances"] > 0
    assert gc["walker_steps"] == oc["walker_steps"]
    assert gc["key_steps"] == oc["key_steps"]
    assert gc["spawn_steps"] == oc["child_steps"]
    for r in range(w.n_replicas):
        _same_store(g.export(r), o.export(r), f"step {w.nsteps} replica {r}")
    # estimators at t_f on the full-size store
    pauli = [(x, z) for _, x, z, _ in w.pauli_obs] + _extra_paulis(w.n, 6, 3)
    _check_observe(g, {r: (o, r) for r in range(w.n_replicas)}, w, pauli, "ghz20_nm t_f")


# ---- dd12 at full size: 121M keys at the end -------------------------------------------------

@pytest.fixture(scope="module")
def dd12_gpu(B):
    """dd12 in the benchmark's launch configuration (automatic path, streamed once the store is
    large, sort tile of 24 records per thread as the autotuner picks on this workload)."""
    w = W.config_dd12()
    g = B.QMC.from_workload(w, store_capacity=1 << 24, spawn_capacity=1 << 21)
    g.tune_sort(24)
    state = {"w": w, "g": g, "step": 0}
    yield state
    g.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("T", [1000, 2000, 3000, 3990])
def test_dd12_imported_states(B, orc, dd12_gpu, T):
    """At step T of the full-size dd12 trajectory every replica is imported into the oracle;
    both then take two steps (T = 1000, 2000, 3000 are pulse steps: the pulse comes first): all
    16 replicas identical.  At T >= 3000 the estimator numerators are compared first."""
    w, g = dd12_gpu["w"], dd12_gpu["g"]
    assert dd12_gpu["step"] <= T
    t0 = time.time()
    g.run_workload(w, dd12_gpu["step"], T)
    dd12_gpu["step"] = T
    R = w.n_replicas
    o = orc.Oracle(w.n, R, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re, w.init_im)
    nk = 0
    for r in range(R):
        k, a, b = g.export(r)
        nk += len(k)
        o.import_(r, k, a, b, step=T)
    _say(f"dd12 step {T}: {nk} keys imported ({time.time() - t0:.1f}s)")
    if T >= 3000:
        pauli = [(x, z) for _, x, z, _ in w.pauli_obs] + _extra_paulis(w.n, 4, T)
        _check_observe(g, {r: (o, r) for r in range(R)}, w, pauli, f"dd12 step {T}")
        _say(f"  estimators equal ({time.time() - t0:.1f}s)")
    for a, b, pulses in w.segments():
        if b <= T or a >= T + 2:
            continue
        if a >= T:
            for (px, pz) in pulses:
                g.pulse(px, pz)
                o.pulse(px, pz)
        lo, hi = max(a, T), min(b, T + 2)
        g.step(w.s[lo:hi], w.gamma[lo:hi])
        o.step(w.s[lo:hi], w.gamma[lo:hi], threads=16)
    dd12_gpu["step"] = T + 2
    for r in range(R):
        _same_store(g.export(r), o.export(r), f"dd12 step {T + 2} replica {r}")
    _say(f"  step {T + 2}: all {R} replicas equal ({time.time() - t0:.1f}s)")
    o.close()


# ---- batch64 at full size: all 64 circuits ---------------------------------------------------

@pytest.fixture(scope="module")
def batch64_gpu(B):
    """The batched configuration in the benchmark's launch configuration (automatic path)."""
    bw = W.config_batch64()
    circuits = [(w.h, w.lops, w.init_keys, w.init_re, w.init_im) for w in bw.circuits]
    g = B.QMC.batch(bw.n, bw.n_replicas, bw.seed, bw.dt, circuits, store_capacity=1 << 18,
                    spawn_capacity=1 << 18)
    g.tune_sort(24)
    state = {"bw": bw, "g": g, "step": 0, "circuits": circuits}
    yield state
    g.close()


def _run_batch(g, bw, start, stop, orcs=None):
    for a, b, masks in bw.segments():
        if b <= start or a >= stop:
            continue
        if a >= start and masks is not None:
            g.pulse_batch(*masks)
            if orcs is not None:
                for c, o in enumerate(orcs):
                    if masks[0][c] or masks[1][c]:
                        o.pulse(int(masks[0][c]), int(masks[1][c]))
        lo, hi = max(a, start), min(b, stop)
        s, gam = bw.weights(lo, hi)
        g.step(s, gam)
        if orcs is not None:
            for o, w in zip(orcs, bw.circuits):
                o.step(w.s[lo:hi], w.gamma[lo:hi], threads=4)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("T", [500, 990])
def test_batch64_imported_states(B, orc, batch64_gpu, T):
    """At step T of the batched configuration every circuit's replicas are imported into an
    oracle of that circuit (its replicas' stream ids c R + r); both take three steps: all 64
    circuits x 4 replicas identical, and the estimator numerators equal before the steps."""
    bw, g = batch64_gpu["bw"], batch64_gpu["g"]
    assert batch64_gpu["step"] <= T
    t0 = time.time()
    _run_batch(g, bw, batch64_gpu["step"], T)
    batch64_gpu["step"] = T
    R = bw.n_replicas
    orcs = []
    for c, (h, lops, keys, re, im) in enumerate(batch64_gpu["circuits"]):
        o = orc.Oracle(bw.n, R, bw.seed, bw.dt, h, lops, keys, re, im)
        o.set_replica_base(c * R)
        for r in range(R):
            o.import_(r, *g.export(c * R + r), step=T)
        orcs.append(o)
    _say(f"batch64 step {T}: {g.counters()['n_occ']} keys imported ({time.time() - t0:.1f}s)")
    # estimators: numerators need no table, so one call covers every circuit
    got = g.observe(pauli=[(0, 1), (1, 0), (3, 3)], want_eps=True)
    for c, o in enumerate(orcs):
        for r in range(R):
            ref = o.observe(r, [(0, 1), (1, 0), (3, 3)])
            seg = c * R + r
            assert int(got["n_occ"][seg]) == ref["n_occ"]
            assert int(got["n_tot"][seg]) == ref["n_tot"]
            assert tuple(got["ndiag"][seg]) == ref["ndiag_int"]
            assert np.array_equal(got["pauli"][seg], ref["pauli"])
            assert got["eps2_int"][seg] == ref["eps2"]
    _run_batch(g, bw, T, T + 3, orcs)
    batch64_gpu["step"] = T + 3
    for c, o in enumerate(orcs):
        for r in range(R):
            _same_store(g.export(c * R + r), o.export(r), f"step {T + 3} circuit {c} replica {r}")
        o.close()
    _say(f"  step {T + 3}: all {len(orcs)} circuits equal ({time.time() - t0:.1f}s)")
