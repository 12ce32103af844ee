"""GPU parity of the learned proposal's deeper network (proposal kind 4: 2n key bits and the step's
active weight channels into two int8 MFMA hidden layers of 128 units): the HIP streamed step
through the C ABI against the CPU oracle, bit for bit, on seeded synthetic inputs and random
(untrained) networks."""
import sys

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


def _same(g, o, R, where):
    for r in range(R):
        for x, y in zip(g.export(r), o.export(r)):
            assert np.array_equal(x, y), f"{where} replica {r}"


@pytest.mark.parametrize("K", [1, 4])
@pytest.mark.parametrize("seed", range(3))
def test_deep_random_models_every_step(B, orc, K, seed):
    """Random models whose weights are zero at some steps (the network's channel inputs change
    from step to step), one and three steps per call."""
    rng = np.random.default_rng(1700 + seed)
    n = int(rng.integers(1, 5))
    h, lops = W.random_model(n, rng, n_h=int(rng.integers(1, 6)), n_l=int(rng.integers(0, 4)))
    R = int(rng.integers(1, 4))
    keys, re, im = W.random_records(n, rng, int(rng.integers(1, 12)), scale=300)
    steps = 6
    s = np.where(rng.random((steps, len(h))) < 0.3, 0.0, rng.normal(size=(steps, len(h))))
    gam = np.where(rng.random((steps, len(lops))) < 0.3, 0.0,
                   np.abs(rng.normal(size=(steps, len(lops)))))
    net = W.random_deep_mlp(rng, s1=2, s2=7)
    _say(f"deep proposal K={K} seed {seed}: n={n} R={R} {len(keys)} keys")
    g = B.QMC(n, R, 50 + seed, 0.01, h, lops, keys, re, im, store_capacity=1 << 12,
              spawn_capacity=1 << 14)
    g.set_path("streamed")
    g.set_proposal_deep(K, net)
    o = orc.Oracle(n, R, 50 + seed, 0.01, h, lops, keys, re, im)
    o.set_proposal_deep(K, net)
    for k in range(3):
        g.step(s[k:k + 1], gam[k:k + 1])
        o.step(s[k:k + 1], gam[k:k + 1])
        _same(g, o, R, f"step {k}")
    g.step(s[3:], gam[3:])
    o.step(s[3:], gam[3:])
    _same(g, o, R, "after the batch")


def test_deep_many_tiles_and_ragged(B, orc):
    rng = np.random.default_rng(1800)
    n, R = 7, 2
    h, lops = W.random_model(n, rng, n_h=8, n_l=3)
    keys = np.arange(1 << (2 * n), dtype=np.uint64)[::3]
    re = rng.integers(-40, 40, size=len(keys)).astype(np.int32)
    im = rng.integers(-40, 40, size=len(keys)).astype(np.int32)
    re[(re == 0) & (im == 0)] = 3
    s = rng.normal(size=(4, len(h))) * 0.3
    gam = np.abs(rng.normal(size=(4, len(lops)))) * 0.3
    net = W.random_deep_mlp(rng, s1=3, s2=8)
    g = B.QMC(n, R, 9, 0.01, h, lops, keys, re, im, store_capacity=1 << 15,
              spawn_capacity=1 << 20)
    g.set_path("streamed")
    g.set_proposal_deep(2, net)
    o = orc.Oracle(n, R, 9, 0.01, h, lops, keys, re, im)
    o.set_proposal_deep(2, net)
    g.step(s, gam)
    o.step(s, gam, threads=2)
    _same(g, o, R, "after 4 steps")


@pytest.mark.timeout(900)
def test_deep_ghz20_nm_all_steps(B, orc):
    """The n=20 GHZ workload with the deeper network over all 3000 steps (two replicas): the GPU
    runs the whole trajectory; its state is imported into the oracle every 250 steps and both
    take three steps from there (the draws are keyed on the walkers, so (store, step) is the whole
    state), and the oracle runs the first 100 steps from the start."""
    w = W.config_ghz20_nm()
    rng = np.random.default_rng(1900)
    net = W.random_deep_mlp(rng, s1=4, s2=9)
    R = 2
    g = B.QMC.from_workload(w, store_capacity=1 << 17, spawn_capacity=1 << 19, n_replicas=R)
    g.set_proposal_deep(2, net)
    o = orc.Oracle(w.n, R, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re, w.init_im)
    o.set_proposal_deep(2, net)
    g.step(w.s[:100], w.gamma[:100])
    o.step(w.s[:100], w.gamma[:100], threads=2)
    _same(g, o, R, "step 100")
    o.close()
    at = 100
    for T in list(range(250, w.nsteps, 250)) + [w.nsteps - 3]:
        g.step(w.s[at:T], w.gamma[at:T])
        o = orc.Oracle(w.n, R, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re, w.init_im)
        o.set_proposal_deep(2, net)
        for r in range(R):
            o.import_(r, *g.export(r), step=T)
        if T == 1500:   # the network is not degenerate here: its scores differ and many are > 0
            act = o.step_active(w.s[T], w.gamma[T])
            sc = np.array([o.deep_scores(int(k), act) for k in g.export(0)[0][:32]])
            assert (sc > 0).mean() > 0.2 and len(np.unique(sc)) > 100
        g.step(w.s[T:T + 3], w.gamma[T:T + 3])
        o.step(w.s[T:T + 3], w.gamma[T:T + 3], threads=2)
        _same(g, o, R, f"steps {T}..{T + 3}")
        _say(f"  deep ghz20_nm steps {T}..{T + 3} equal, {g.counters()['n_occ']} keys")
        o.close()
        at = T + 3
    assert at == w.nsteps


def test_deep_refusals(B):
    rng = np.random.default_rng(2000)
    h, lops = W.random_model(2, rng)
    keys, re, im = W.random_records(2, rng, 4)
    g = B.QMC(2, 1, 1, 0.01, h, lops, keys, re, im, store_capacity=64, spawn_capacity=256)
    net = W.random_deep_mlp(rng)
    for K in (0, 3, 128):
        with pytest.raises(B.QMCError) as e:
            g.set_proposal_deep(K, net)
        assert e.value.code == B.QMC_ERR_ARG
    bad = list(net)
    bad[7] = 31
    with pytest.raises(B.QMCError) as e:
        g.set_proposal_deep(2, tuple(bad))
    assert e.value.code == B.QMC_ERR_ARG
    with pytest.raises(ValueError):
        g.set_proposal_deep(2, (net[0][:64],) + tuple(net[1:]))
    g.set_proposal_deep(2, net)
    with pytest.raises(B.QMCError):
        g.set_integrator("ab2")
    with pytest.raises(B.QMCError):
        g.set_initiator(10)
    g.set_proposal("comb")
    g.set_initiator(10)
    with pytest.raises(B.QMCError) as e:
        g.set_proposal_deep(2, net)
    assert e.value.code == B.QMC_ERR_ARG


def test_spawn_log_holds_the_plain_children(B, orc):
    """The spawn-event log of a plain streamed run: one event per nonzero off-diagonal child, as
    many as the oracle's child records over the same steps, each naming a column group of its
    step's table and a parent of that step; logging changes no result; a full buffer keeps
    counting."""
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    g.log_spawns(1 << 16)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    parents = {}
    for k in range(60):
        parents[k] = {int(key) | (r << (2 * w.n)) for r in range(w.n_replicas)
                      for key in g.export(r)[0]}
        g.step(w.s[k:k + 1], w.gamma[k:k + 1])
        o.step(w.s[k:k + 1], w.gamma[k:k + 1])
    _same(g, o, w.n_replicas, "step 60 with logging")
    ev, total = g.log_read()
    assert total == len(ev) == o.counters()["child_steps"] == g.counters()["spawn_steps"]
    assert np.all((ev["re"] != 0) | (ev["im"] != 0))
    for k in range(60):
        sel = ev[ev["step"] == k]
        G = len(B.coeff_table(w.n, w.dt, w.h, w.lops, w.s[k], w.gamma[k])["gxmask"])
        assert np.all((sel["group"] >= 1) & (sel["group"] < G))
        assert {int(x) for x in sel["key"]} <= parents[k]
    g.log_spawns(10)
    g.step(w.s[60:80], w.gamma[60:80])
    ev2, total2 = g.log_read()
    assert len(ev2) == 10 and total2 > 10
    g.log_spawns(0)
    g.step(w.s[80:90], w.gamma[80:90])
