"""GPU parity of the LDS-resident step (one workgroup per replica, a whole batch of steps per
launch, for stores of at most 2048 keys per replica) against the oracle: whole stores bit for bit
after every call, on the forced path and inside the automatic one, including the hand-over to
the fused kernel when a replica outgrows it."""
import numpy as np
import pytest

from paper_2502_18929_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_18929_amd import binding
    binding.lib()
    return binding


def _same(g, o, R, where):
    for r in range(R):
        for x, y in zip(g.export(r), o.export(r)):
            assert np.array_equal(x, y), f"{where} replica {r}"


@pytest.mark.parametrize("seed", range(5))
def test_small_random_models_every_step(B, orc, seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(1, 5))
    h, lops = W.random_model(n, rng, n_h=int(rng.integers(1, 6)), n_l=int(rng.integers(0, 4)))
    keys, re, im = W.random_records(n, rng, int(rng.integers(1, 12)), scale=300)
    R = int(rng.integers(1, 6))
    g = B.QMC(n, R, 40 + seed, 0.02, h, lops, keys, re, im, store_capacity=256,
              spawn_capacity=4096)
    g.set_path("small")
    o = orc.Oracle(n, R, 40 + seed, 0.02, h, lops, keys, re, im)
    s = rng.uniform(-1, 1, size=(60, len(h)))
    gam = rng.uniform(-0.2, 0.6, size=(60, len(lops)))
    for a in (0, 1, 7, 30):
        b = {0: 1, 1: 7, 7: 30, 30: 60}[a]
        g.step(s[a:b], gam[a:b])
        o.step(s[a:b], gam[a:b])
        _same(g, o, R, f"seed {seed} step {b}")
    assert g.counters()["walker_steps"] == o.counters()["walker_steps"]
    assert g.counters()["spawn_steps"] == o.counters()["child_steps"]


def test_small_ghz4_whole_trajectory(B, orc):
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    g.set_path("small")
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    g.step(w.s, w.gamma)
    o.step(w.s, w.gamma)
    _same(g, o, w.n_replicas, "ghz4 step 400")


def test_small_initiator_and_shift(B, orc):
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    g.set_path("small")
    g.set_initiator(40)
    g.set_shift(1, 0.7)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    o.set_initiator(40)
    o.set_shift(1, 0.7)
    for a in range(0, 400, 80):
        g.step(w.s[a:a + 80], w.gamma[a:a + 80])
        o.step(w.s[a:a + 80], w.gamma[a:a + 80])
        _same(g, o, w.n_replicas, f"step {a + 80}")


def test_small_batch_of_circuits(B, orc):
    rng = np.random.default_rng(91)
    circuits = []
    for c in range(3):
        h, lops = W.random_model(3, rng, n_h=3, n_l=2)
        keys, re, im = W.random_records(3, rng, 5, scale=200)
        circuits.append((h, lops, keys, re, im))
    R = 2
    g = B.QMC.batch(3, R, 13, 0.01, circuits, store_capacity=64, spawn_capacity=2048)
    g.set_path("small")
    orcs = []
    for c, (h, lops, keys, re, im) in enumerate(circuits):
        o = orc.Oracle(3, R, 13, 0.01, h, lops, keys, re, im)
        o.set_replica_base(c * R)
        orcs.append(o)
    s = [rng.uniform(-1, 1, size=(40, len(c[0]))) for c in circuits]
    gam = [rng.uniform(0.0, 0.4, size=(40, len(c[1]))) for c in circuits]
    g.step(np.concatenate(s, axis=1), np.concatenate(gam, axis=1))
    for c, o in enumerate(orcs):
        o.step(s[c], gam[c])
        for r in range(R):
            for x, y in zip(g.export(c * R + r), o.export(r)):
                assert np.array_equal(x, y), (c, r)


@pytest.mark.timeout(600)
def test_small_hands_over_to_the_fused_kernel(B, orc):
    """ghz20_nm in the automatic mode: the LDS-resident step carries the first steps, a replica
    outgrows its key limit, the fused kernel takes the rest; compared with the oracle every 250
    steps, and the small path forced past its capacity reports the store error."""
    w = W.config_ghz20_nm()
    g = B.QMC.from_workload(w, store_capacity=1 << 17, spawn_capacity=1 << 19)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    g.profile("small")
    for a in range(0, w.nsteps, 250):
        g.step(w.s[a:a + 250], w.gamma[a:a + 250])
        o.step(w.s[a:a + 250], w.gamma[a:a + 250], threads=16)
        _same(g, o, w.n_replicas, f"step {a + 250}")
    ms, n, cov = g.profile_read()
    assert n > 0 and 0 < cov["steps"] < w.nsteps
    _, nf, covf = g.profile_read("fused")
    assert nf > 0 and cov["steps"] + covf["steps"] == w.nsteps
    gc, oc = g.counters(), o.counters()
    assert gc["walker_steps"] == oc["walker_steps"] and gc["key_steps"] == oc["key_steps"]
    assert gc["spawn_steps"] == oc["child_steps"]
    h = B.QMC.from_workload(w, store_capacity=1 << 17, spawn_capacity=1 << 19)
    h.set_path("small")
    with pytest.raises(B.QMCError) as e:
        h.step(w.s, w.gamma)
    assert e.value.code == B.QMC_ERR_STORE_CAP


@pytest.mark.timeout(600)
def test_small_limits_change_nothing(B, orc):
    """One call over the whole ghz20_nm trajectory (a chain of 64-step batches that stops
    inside a batch, which is run again up to the stop) at several key limits, and with the
    LDS-resident step off: the same final stores as the oracle, the same counters."""
    w = W.config_ghz20_nm()
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    o.step(w.s, w.gamma, threads=16)
    oc = o.counters()
    covered = {}
    for lim in (0, 37, 300, 1024):
        g = B.QMC.from_workload(w, store_capacity=1 << 17, spawn_capacity=1 << 19)
        g.small_limit(lim)
        g.profile("small")
        g.step(w.s, w.gamma)
        _same(g, o, w.n_replicas, f"limit {lim}")
        gc = g.counters()
        assert gc["walker_steps"] == oc["walker_steps"] and gc["key_steps"] == oc["key_steps"]
        covered[lim] = g.profile_read()[2]["steps"]
        g.close()
    assert covered[0] == 0 < covered[37] < covered[300] <= covered[1024] < w.nsteps
    with pytest.raises(B.QMCError) as e:
        g = B.QMC.from_workload(w, store_capacity=1 << 17, spawn_capacity=1 << 19)
        g.small_limit(1025)
    assert e.value.code == B.QMC_ERR_ARG


@pytest.mark.timeout(600)
@pytest.mark.parametrize("lim", [4, 16, 60])
def test_small_head_batch_calls(B, orc, lim):
    """Calls of 8 to 511 steps, whose first batch is launched while the rest of the call's tables
    are built, on ghz20_nm with key limits that stop the chain inside that first batch or in a
    later one (the steps up to the stop are run again, the rest go to the fused kernel): the
    stores equal the oracle's after every call, and so do the counters."""
    w = W.config_ghz20_nm()
    g = B.QMC.from_workload(w, store_capacity=1 << 17, spawn_capacity=1 << 19)
    g.small_limit(lim)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    g.profile("small")
    a = 0
    for k in (8, 9, 20, 37, 100, 200, 511):
        g.step(w.s[a:a + k], w.gamma[a:a + k])
        o.step(w.s[a:a + k], w.gamma[a:a + k], threads=16)
        a += k
        _same(g, o, w.n_replicas, f"limit {lim}, step {a}")
    ms, n, cov = g.profile_read()
    assert n > 0 and 0 < cov["steps"] < a
    gc, oc = g.counters(), o.counters()
    assert gc["walker_steps"] == oc["walker_steps"] and gc["key_steps"] == oc["key_steps"]
    assert gc["spawn_steps"] == oc["child_steps"]


def test_small_head_batch_cancelled_by_a_later_table(B, orc):
    """A bad weight in a table built after the first batch was launched: the call fails naming
    that step, and the store and counters are those before the call."""
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    g.step(w.s[:10], w.gamma[:10])
    o.step(w.s[:10], w.gamma[:10])
    before = g.counters()
    s = np.array(w.s[10:50])
    s[30, 0] = np.nan
    with pytest.raises(B.QMCError) as e:
        g.step(s, w.gamma[10:50])
    assert e.value.code == B.QMC_ERR_ARG and "step 40" in str(e.value)
    _same(g, o, w.n_replicas, "after the failed call")
    assert g.counters() == before
    g.step(w.s[10:50], w.gamma[10:50])
    o.step(w.s[10:50], w.gamma[10:50])
    _same(g, o, w.n_replicas, "step 50")
