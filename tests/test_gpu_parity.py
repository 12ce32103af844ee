"""GPU parity: the HIP step through the C ABI against the CPU oracle, bit for bit.

Every comparison is of whole per-replica stores (sorted keys, int32 re, int32 im) after a step
or a batch of steps, on seeded synthetic inputs; both sides run their own trajectories from the
same initial records (nothing flows from the GPU into the oracle).
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


PATHS = ["fused", "streamed"]


def _pair(B, orc, w, R=None, store=None, spawn=None, seed=None, path="auto"):
    R = w.n_replicas if R is None else R
    seed = w.seed if seed is None else seed
    g = B.QMC.from_workload(w, store_capacity=store, spawn_capacity=spawn, n_replicas=R,
                            seed=seed)
    g.set_path(path)
    o = orc.Oracle(w.n, R, seed, w.dt, w.h, w.lops, w.init_keys, w.init_re, w.init_im)
    return g, o


def _assert_same(g, o, R, where=""):
    for r in range(R):
        gk, ga, gb = g.export(r)
        ok, oa, ob = o.export(r)
        if not (np.array_equal(gk, ok) and np.array_equal(ga, oa) and np.array_equal(gb, ob)):
            n = min(len(gk), len(ok))
            bad = np.nonzero((gk[:n] != ok[:n]) | (ga[:n] != oa[:n]) | (gb[:n] != ob[:n]))[0]
            first = int(bad[0]) if len(bad) else n
            raise AssertionError(f"{where} replica {r}: sizes gpu {len(gk)} oracle {len(ok)}, "
                                 f"first difference at {first}: gpu "
                                 f"{(gk[first:first+1], ga[first:first+1], gb[first:first+1])} "
                                 f"oracle {(ok[first:first+1], oa[first:first+1], ob[first:first+1])}")


def _run_both(g, o, w, start, stop, threads=1):
    for a, b, pulses in w.segments():
        if b <= start or a >= stop:
            continue
        if a >= start:
            for (px, pz) in pulses:
                g.pulse(px, pz)
                o.pulse(px, pz)
        lo, hi = max(a, start), min(b, stop)
        g.step(w.s[lo:hi], w.gamma[lo:hi])
        o.step(w.s[lo:hi], w.gamma[lo:hi], threads=threads)


# ---- small random models: every step, several replicas --------------------------------------

@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(6))
def test_random_models_every_step(B, orc, seed, path):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 5))
    h, lops = W.random_model(n, rng, n_h=int(rng.integers(1, 6)), n_l=int(rng.integers(0, 4)))
    keys, re, im = W.random_records(n, rng, int(rng.integers(1, 12)), scale=3000)
    R = int(rng.integers(1, 5))
    dt = 0.01
    _say(f"random model seed={seed} n={n} R={R} keys={len(keys)} path={path}")
    g = B.QMC(n, R, 1000 + seed, dt, h, lops, keys, re, im, store_capacity=1 << (2 * n),
              spawn_capacity=4096)
    g.set_path(path)
    o = orc.Oracle(n, R, 1000 + seed, dt, h, lops, keys, re, im)
    s = rng.normal(size=(40, len(h))) * 0.5
    gam = np.abs(rng.normal(size=(40, len(lops)))) * 0.5
    for k in range(40):
        g.step(s[k:k + 1], gam[k:k + 1])
        o.step(s[k:k + 1], gam[k:k + 1])
        _assert_same(g, o, R, f"step {k}")


@pytest.mark.parametrize("path", PATHS)
def test_ghz4_full_trajectory(B, orc, path):
    w = W.config_ghz4()
    _say(f"{w.name}: {w.nsteps} steps x {w.n_replicas} replicas, {path}")
    g, o = _pair(B, orc, w, store=256, spawn=4096, path=path)
    for k0 in range(0, w.nsteps, 20):
        _run_both(g, o, w, k0, k0 + 20)
        _assert_same(g, o, w.n_replicas, f"step {k0 + 20}")
    c = g.counters()
    assert c["step"] == w.nsteps


@pytest.mark.parametrize("path", PATHS)
def test_multi_tile_ragged_one_step(B, orc, path):
    """Thousands of keys spread over many merge tiles and a ragged tail."""
    rng = np.random.default_rng(9)
    n = 7
    h, lops = W.random_model(n, rng, n_h=6, n_l=3)
    for count in (1, 1023, 1024, 1025, 5000, 12289):
        keys, re, im = W.random_records(n, rng, count, scale=200)
        R = 3
        _say(f"multi-tile one step: {count} keys x {R} replicas, {path}")
        g = B.QMC(n, R, 7, 0.01, h, lops, keys, re, im, store_capacity=1 << 14,
                  spawn_capacity=1 << 20)
        g.set_path(path)
        o = orc.Oracle(n, R, 7, 0.01, h, lops, keys, re, im)
        s = rng.normal(size=(3, len(h)))
        gam = np.abs(rng.normal(size=(3, len(lops))))
        for k in range(3):
            g.step(s[k:k + 1], gam[k:k + 1])
            o.step(s[k:k + 1], gam[k:k + 1])
            _assert_same(g, o, R, f"count {count} step {k}")
        g.close()


@pytest.mark.parametrize("path", PATHS)
def test_dd_small_with_pulses(B, orc, path):
    w = W.dd(n=6, n_replicas=4, walker_target=20000, nsteps=800, seed=11)
    _say(f"dd n=6: {w.nsteps} steps with ideal pulses, {path}")
    g, o = _pair(B, orc, w, store=4096, spawn=1 << 16, path=path)
    for k0 in range(0, w.nsteps, 100):
        _run_both(g, o, w, k0, k0 + 100)
        _assert_same(g, o, w.n_replicas, f"step {k0 + 100}")


@pytest.mark.parametrize("path", PATHS)
def test_dd_small_finite_pulses(B, orc, path):
    """DD with square pulses of width 0.05 integrated with steps of dt / 10 inside them (weights
    and rates divided by 10 there): three pulse windows, the last completed past the run."""
    w = W.dd(n=6, n_replicas=4, walker_target=20000, nsteps=300, seed=12, pulse_width=0.05,
             substeps=10)
    _say(f"dd n=6: {w.nsteps} steps with finite pulses, {path}")
    g, o = _pair(B, orc, w, store=4096, spawn=1 << 16, path=path)
    for k0 in range(0, w.nsteps, 150):
        _run_both(g, o, w, k0, min(k0 + 150, w.nsteps))
        _assert_same(g, o, w.n_replicas, f"step {min(k0 + 150, w.nsteps)}")


def test_general_pauli_pulse_resorts(B, orc):
    rng = np.random.default_rng(4)
    n = 5
    keys, re, im = W.random_records(n, rng, 300, scale=1000)
    g = B.QMC(n, 2, 1, 0.01, [], [], keys, re, im, store_capacity=1024, spawn_capacity=1024)
    o = orc.Oracle(n, 2, 1, 0.01, [], [], keys, re, im)
    for x, z in [(0, 3), (5, 0), (31, 17), (1, 1)]:
        g.pulse(x, z)
        o.pulse(x, z)
        _assert_same(g, o, 2, f"pulse {x},{z}")


# ---- the three configurations at full size ---------------------------------------------------

@pytest.mark.parametrize("path", ["auto", "streamed"])
def test_ghz20_nm_full_size(B, orc, path):
    """n=20 non-Markovian GHZ, 8 replicas x 1e7 walkers, all 3000 steps (the benchmarked
    workload, same launch configuration), every replica compared every 250 steps."""
    w = W.config_ghz20_nm()
    _say(f"{w.name}: full size {w.nsteps} steps x {w.n_replicas} replicas, {path}")
    g, o = _pair(B, orc, w, store=1 << 17, spawn=1 << 19, path=path)
    t0 = time.time()
    for k0 in range(0, w.nsteps, 250):
        g.step(w.s[k0:k0 + 250], w.gamma[k0:k0 + 250])
        o.step(w.s[k0:k0 + 250], w.gamma[k0:k0 + 250], threads=16)
        _assert_same(g, o, w.n_replicas, f"step {k0 + 250}")
        _say(f"  step {k0 + 250} equal ({time.time() - t0:.1f}s)")
    # the growing population made the fused kernel re-cut its key ranges (inside its launches)
    reb = g.counters()["rebalances"]
    _say(f"  key-range re-cuts: {reb}")
    assert (reb > 0) == (path == "auto")


@pytest.mark.parametrize("path", PATHS)
def test_dd12_full_size_first_steps(B, orc, path):
    """n=12 DD at full size (16 replicas x 1e6 walkers) over the first 600 steps (five pulse
    times), every replica against the oracle."""
    w = W.config_dd12()
    _say(f"{w.name}: 16 replicas, first 600 steps, {path}")
    g = B.QMC.from_workload(w, store_capacity=1 << 20, spawn_capacity=1 << 18)
    g.set_path(path)
    o = orc.Oracle(w.n, 16, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re, w.init_im)
    _run_both(g, o, w, 0, 600, threads=16)
    _assert_same(g, o, 16, "step 600")


def test_whole_step_timing_changes_nothing(B, orc):
    """Timing whole streamed steps (class 'step', which times the merge class beside it) covers
    exactly the steps run, in chunks, and leaves the stores equal to the oracle's."""
    w = W.config_dd12()
    g = B.QMC.from_workload(w, store_capacity=1 << 20, spawn_capacity=1 << 18)
    g.set_path("streamed")
    o = orc.Oracle(w.n, 16, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re, w.init_im)
    g.profile("step")
    _run_both(g, o, w, 0, 300, threads=16)
    _assert_same(g, o, 16, "step 300")
    ms, n, cov = g.profile_read()
    assert cov["steps"] == 300 and 1 <= n < 300 and ms > 0
    ms2, n2, cov2 = g.profile_read("merge")
    assert n2 == 300 and cov2 == cov and 0 < ms2 < ms
    oc = o.counters()
    assert cov["walker_steps"] == oc["walker_steps"] and cov["key_steps"] == oc["key_steps"]
    g.profile(None)


# ---- estimators ------------------------------------------------------------------------------

def test_observe_matches_oracle(B, orc):
    w = W.config_ghz4()
    g, o = _pair(B, orc, w, store=256, spawn=4096)
    _run_both(g, o, w, 0, 260)
    pauli = [(x, z) for _, x, z, _ in w.pauli_obs] + [(3, 5), (15, 15), (0, 0)]
    got = g.observe(pauli=pauli, psi=w.psi, want_eps=True)
    lk = [(v << w.n) | u for u, _ in w.psi for v, _ in w.psi]
    for r in range(w.n_replicas):
        ref = o.observe(r, pauli, lk)
        assert int(got["n_occ"][r]) == ref["n_occ"]
        assert int(got["n_tot"][r]) == ref["n_tot"]
        assert tuple(got["ndiag"][r]) == ref["ndiag_int"]
        assert np.array_equal(got["pauli"][r], ref["pauli"])
        assert got["eps2_int"][r] == ref["eps2"]
        nd0 = float(w.walker_target)
        F = 0.0
        idx = 0
        for u, au in w.psi:
            for v, av in w.psi:
                F += (np.conj(au) * av * complex(*ref["lookup"][idx])).real
                idx += 1
        assert abs(got["fidelity"][r, 0] - F / nd0) < 1e-12
        assert got["trace"][r] == ref["ndiag_int"][0] / nd0


# ---- invariances and failure handling --------------------------------------------------------

def test_replica_count_invariance(B, orc):
    w = W.config_ghz4()
    a = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096, n_replicas=2)
    b = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096, n_replicas=7)
    a.step(w.s[:200], w.gamma[:200])
    b.step(w.s[:200], w.gamma[:200])
    for r in range(2):
        for x, y in zip(a.export(r), b.export(r)):
            assert np.array_equal(x, y)


def test_export_import_resume(B, orc):
    w = W.config_ghz4()
    a = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    a.step(w.s[:300], w.gamma[:300])
    b = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    b.step(w.s[:150], w.gamma[:150])
    c = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    for r in range(w.n_replicas):
        c.import_(r, *b.export(r), step=150)
    c.step(w.s[150:300], w.gamma[150:300])
    for r in range(w.n_replicas):
        for x, y in zip(a.export(r), c.export(r)):
            assert np.array_equal(x, y)


def test_empty_replica_stays_empty(B, orc):
    w = W.config_ghz4()
    g, o = _pair(B, orc, w, store=256, spawn=4096)
    e = np.zeros(0, np.uint64), np.zeros(0, np.int32), np.zeros(0, np.int32)
    g.import_(1, *e, step=0)
    o.import_(1, *e, step=0)
    _run_both(g, o, w, 0, 120)
    _assert_same(g, o, w.n_replicas, "empty replica")
    assert len(g.export(1)[0]) == 0


@pytest.mark.parametrize("path", PATHS)
def test_spawn_capacity_error_rolls_back(B, orc, path):
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=2)
    g.set_path(path)
    with pytest.raises(B.QMCError) as e:
        g.step(w.s[:50], w.gamma[:50])
    assert e.value.code == B.QMC_ERR_SPAWN_CAP
    st = g.counters()["step"]
    snap = [g.export(r) for r in range(w.n_replicas)]
    # retry that step with enough capacity: identical to an uninterrupted run
    big = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    for r in range(w.n_replicas):
        big.import_(r, *snap[r], step=st)
    big.step(w.s[st:60], w.gamma[st:60])
    ref = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    ref.step(w.s[:60], w.gamma[:60])
    for r in range(w.n_replicas):
        for x, y in zip(big.export(r), ref.export(r)):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("path", PATHS)
def test_store_capacity_error(B, orc, path):
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=3, spawn_capacity=4096)
    g.set_path(path)
    with pytest.raises(B.QMCError) as e:
        g.step(w.s[:400], w.gamma[:400])
    assert e.value.code == B.QMC_ERR_STORE_CAP
    st = g.counters()["step"]
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    o.step(w.s[:st], w.gamma[:st])
    _assert_same(g, o, w.n_replicas, "rolled back")


@pytest.mark.parametrize("path", PATHS)
def test_count_overflow_error(B, orc, path):
    g = B.QMC(1, 1, 1, 0.01, [], [], [0], [2_000_000_000], [0], store_capacity=4,
              spawn_capacity=4)
    g.set_path(path)
    g.set_shift(0, 20.0)
    with pytest.raises(B.QMCError) as e:
        g.step(np.zeros((1, 0)), np.zeros((1, 0)))
    assert e.value.code == B.QMC_ERR_COUNT_OVERFLOW
    k, a, b = g.export(0)
    assert a[0] == 2_000_000_000 and g.counters()["step"] == 0


def test_shift_matches_oracle(B, orc):
    w = W.config_ghz4()
    g, o = _pair(B, orc, w, store=256, spawn=4096)
    for r in range(w.n_replicas):
        g.set_shift(r, 0.3 * (r - 1.5))
        o.set_shift(r, 0.3 * (r - 1.5))
    _run_both(g, o, w, 0, 100)
    _assert_same(g, o, w.n_replicas, "shifted")


def _dense_spawner(n=8, R=4, seed=21):
    """Every key of an n-qubit register occupied, with a model of many column groups: each key
    range of the fused kernel receives far more than one inbox of children per step."""
    rng = np.random.default_rng(seed)
    h, lops = W.random_model(n, rng, n_h=24, n_l=4)
    keys = np.arange(1 << (2 * n), dtype=np.uint64)
    re = rng.integers(-3000, 3000, size=len(keys)).astype(np.int32)
    im = rng.integers(-3000, 3000, size=len(keys)).astype(np.int32)
    re[(re == 0) & (im == 0)] = 1
    s = rng.normal(size=(3, len(h)))
    gam = np.abs(rng.normal(size=(3, len(lops))))
    return n, R, h, lops, keys, re, im, s, gam


@pytest.mark.parametrize("n_h", [6, 16])
def test_fused_large_inboxes(B, orc, n_h):
    """Every key of an n=7 register occupied (16384 keys) under a model of ~2*n_h column groups:
    each key range of the fused kernel receives about a thousand (n_h=6) to a few thousand
    (n_h=16) records per step, so the inbox sorts beyond 512 and 1024 records run."""
    rng = np.random.default_rng(40 + n_h)
    n, R = 7, 1
    h, lops = W.random_model(n, rng, n_h=n_h, n_l=2)
    keys = np.arange(1 << (2 * n), dtype=np.uint64)
    re = rng.integers(-3000, 3000, size=len(keys)).astype(np.int32)
    im = rng.integers(-3000, 3000, size=len(keys)).astype(np.int32)
    re[(re == 0) & (im == 0)] = 1
    s = rng.normal(size=(3, len(h))) * 0.5
    gam = np.abs(rng.normal(size=(3, len(lops)))) * 0.5
    _say(f"fused large inboxes: n_h={n_h}, {len(keys)} keys")
    g = B.QMC(n, R, 11, 0.01, h, lops, keys, re, im, store_capacity=1 << 15,
              spawn_capacity=1 << 22)
    g.set_path("fused")
    o = orc.Oracle(n, R, 11, 0.01, h, lops, keys, re, im)
    for k in range(3):
        g.step(s[k:k + 1], gam[k:k + 1])
        o.step(s[k:k + 1], gam[k:k + 1])
        _assert_same(g, o, R, f"n_h={n_h} step {k}")
    c = g.counters()
    _say(f"  routed records per key range per step: {c['child_steps'] / 3 / 256:.0f}")


def test_auto_path_falls_back_to_streamed(B, orc):
    n, R, h, lops, keys, re, im, s, gam = _dense_spawner()
    _say(f"dense spawner: {len(keys)} keys x {R} replicas, automatic path")
    g = B.QMC(n, R, 5, 0.01, h, lops, keys, re, im, store_capacity=1 << 17,
              spawn_capacity=1 << 23)
    o = orc.Oracle(n, R, 5, 0.01, h, lops, keys, re, im)
    g.step(s, gam)
    o.step(s, gam, threads=8)
    _assert_same(g, o, R, "after 3 steps")


def test_fused_only_reports_inbox_overflow(B, orc):
    n, R, h, lops, keys, re, im, s, gam = _dense_spawner()
    g = B.QMC(n, R, 5, 0.01, h, lops, keys, re, im, store_capacity=1 << 17,
              spawn_capacity=1 << 23)
    g.set_path("fused")
    with pytest.raises(B.QMCError) as e:
        g.step(s, gam)
    assert e.value.code == B.QMC_ERR_SPAWN_CAP
    st = g.counters()["step"]
    o = orc.Oracle(n, R, 5, 0.01, h, lops, keys, re, im)
    o.step(s[:st], gam[:st])
    _assert_same(g, o, R, f"rolled back to step {st}")


def test_dt_error_leaves_state(B, orc):
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    g.step(w.s[:10], w.gamma[:10])
    before = g.export(0)
    with pytest.raises(B.QMCError) as e:
        g.step(w.s[10:11] * 1e4, w.gamma[10:11])
    assert e.value.code == B.QMC_ERR_DT
    after = g.export(0)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert g.counters()["step"] == 10


@pytest.mark.parametrize("path", PATHS)
def test_call_longer_than_one_table_window(B, orc, path):
    """8500 steps in one call: the tables come in two windows (at most 8000 steps each)."""
    rng = np.random.default_rng(77)
    n = 2
    h, lops = W.random_model(n, rng, n_h=3, n_l=2)
    keys, re, im = W.random_records(n, rng, 5, scale=2000)
    N = 8500
    s = np.cos(np.arange(N) / 300.0)[:, None] * np.ones((1, len(h)))
    gam = np.abs(np.sin(np.arange(N) / 500.0))[:, None] * np.ones((1, len(lops)))
    _say(f"8500-step call, {path}")
    g = B.QMC(n, 2, 31, 0.002, h, lops, keys, re, im, store_capacity=64, spawn_capacity=4096)
    g.set_path(path)
    o = orc.Oracle(n, 2, 31, 0.002, h, lops, keys, re, im)
    g.step(s, gam)
    o.step(s, gam)
    for r in range(2):
        for x, y in zip(g.export(r), o.export(r)):
            assert np.array_equal(x, y), f"replica {r}"


def test_tables_larger_than_a_staging_slice(B, orc):
    """Every Pauli monomial of n=5 in H (about 2000 terms, 34 KB per table): the host threads'
    staging slices cannot hold all their steps, so the call runs over several table windows."""
    rng = np.random.default_rng(5)
    n = 5
    h = [(x, z, (1j if bin(x & z).count("1") & 1 else 1) * 0.005 * rng.normal())
         for x in range(32) for z in range(32)]
    lops = [[(1 << q, 0, 0.3)] for q in range(n)]
    N = 1024
    s = np.ones((N, len(h))) * (1 + 0.1 * np.sin(np.arange(N) / 50))[:, None]
    gam = np.ones((N, len(lops))) * 0.05
    keys, re, im = W.random_records(n, rng, 8, scale=20)
    _say("dense tables, 1024 steps, streamed")
    g = B.QMC(n, 1, 9, 0.001, h, lops, keys, re, im, store_capacity=1024, spawn_capacity=1 << 16)
    o = orc.Oracle(n, 1, 9, 0.001, h, lops, keys, re, im)
    g.step(s, gam)
    o.step(s, gam)
    for x, y in zip(g.export(0), o.export(0)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("bad, code", [(1, "DT"), (1537, "DT"), (2999, "ARG")])
def test_long_call_table_error_names_first_step(B, orc, bad, code):
    """A 3000-step call builds its tables on several host threads: the first bad step is
    reported (by step number) and nothing runs."""
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    g.step(w.s[:10], w.gamma[:10])
    before = g.export(0)
    s = np.tile(w.s[10:11], (3000, 1))
    gam = np.tile(w.gamma[10:11], (3000, 1))
    if code == "DT":
        s[bad] *= 1e4
        s[2990] *= 1e4  # a later bad step is not the one reported
    else:
        gam[bad, 0] = np.nan
    with pytest.raises(B.QMCError) as e:
        g.step(s, gam)
    assert e.value.code == getattr(B, "QMC_ERR_" + code)
    assert f"step {10 + bad}:" in str(e.value)
    after = g.export(0)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert g.counters()["step"] == 10


def test_dd12_full_size_paths_agree(B):
    """dd12 at full size, all 4000 steps (up to 121M keys), in the benchmark's launch
    configuration (automatic path: fused while the store is small, then streamed with the
    autotuned sort tile) against the streamed path alone with the default tile: every replica
    identical, stores sorted, unique and free of empty records.  (The oracle follows dd12 over
    its first 600 steps above; at 121M keys it would take hours.)"""
    w = W.config_dd12()
    _say(f"{w.name}: full size, {w.nsteps} steps, automatic vs streamed")
    stores = []
    for path, tune in [("auto", 0), ("streamed", 16)]:
        g = B.QMC.from_workload(w, store_capacity=1 << 24, spawn_capacity=1 << 21)
        g.set_path(path)
        g.tune_sort(tune)
        g.run_workload(w, 0, w.nsteps)
        stores.append([g.export(r) for r in range(w.n_replicas)])
        _say(f"  {path}: {g.counters()['n_occ']} keys at the end")
        g.close()
    for r in range(w.n_replicas):
        ka, aa, ba = stores[0][r]
        kb, ab, bb = stores[1][r]
        assert np.array_equal(ka, kb) and np.array_equal(aa, ab) and np.array_equal(ba, bb), r
        assert np.all(ka[1:] > ka[:-1])
        assert not np.any((aa == 0) & (ba == 0))
