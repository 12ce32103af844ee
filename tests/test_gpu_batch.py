"""GPU parity of the batched step (many circuits of different size in one context and one step
launch) against the oracle run circuit by circuit: replica r of circuit c is store segment
c * R + r and draws Philox stream c * R + r, which the oracle reproduces with a replica base.
Whole per-segment stores are compared bit for bit, on both step paths."""
import sys

import numpy as np
import pytest

from paper_2502_18929_amd import workloads as W

pytestmark = pytest.mark.gpu
PATHS = ["fused", "streamed"]


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


def _oracles(orc, n, R, seed, dt, circuits):
    out = []
    for c, (h, lops, keys, re, im) in enumerate(circuits):
        o = orc.Oracle(n, R, seed, dt, h, lops, keys, re, im)
        o.set_replica_base(c * R)
        out.append(o)
    return out


def _same(g, oracles, R, where):
    for c, o in enumerate(oracles):
        for r in range(R):
            for a, b in zip(g.export(c * R + r), o.export(r)):
                if not np.array_equal(a, b):
                    raise AssertionError(f"{where}: circuit {c} replica {r}")


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(3))
def test_batch_random_circuits_every_step(B, orc, seed, path):
    rng = np.random.default_rng(1200 + seed)
    n = 5
    C = int(rng.integers(2, 7))
    R = int(rng.integers(1, 4))
    circuits = []
    for c in range(C):
        nc = int(rng.integers(1, n + 1))
        h, lops = W.random_model(nc, rng, n_h=int(rng.integers(0, 6)),
                                 n_l=int(rng.integers(0, 4)))
        keys, re, im = W.random_records(nc, rng, int(rng.integers(1, 8)), scale=500)
        circuits.append((h, lops, keys, re, im))
    _say(f"batch seed={seed} C={C} R={R} path={path}")
    g = B.QMC.batch(n, R, 40 + seed, 0.01, circuits, store_capacity=1 << (2 * n),
                    spawn_capacity=1 << 14)
    g.set_path(path)
    orcs = _oracles(orc, n, R, 40 + seed, 0.01, circuits)
    steps = 30
    ws = [(rng.normal(size=(steps, len(h))), np.abs(rng.normal(size=(steps, len(l)))))
          for (h, l, _, _, _) in circuits]
    s_all = np.concatenate([w[0] for w in ws], axis=1)
    g_all = np.concatenate([w[1] for w in ws], axis=1)
    for k in range(steps):
        g.step(s_all[k:k + 1], g_all[k:k + 1])
        for c, o in enumerate(orcs):
            o.step(ws[c][0][k:k + 1], ws[c][1][k:k + 1])
        _same(g, orcs, R, f"step {k}")


@pytest.mark.parametrize("path", PATHS)
def test_batch_of_one_circuit_is_the_plain_context(B, orc, path):
    w = W.config_ghz4()
    a = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=8192)
    b = B.QMC.batch(w.n, w.n_replicas, w.seed, w.dt,
                    [(w.h, w.lops, w.init_keys, w.init_re, w.init_im)], store_capacity=256,
                    spawn_capacity=8192)
    a.set_path(path)
    b.set_path(path)
    a.step(w.s, w.gamma)
    b.step(w.s, w.gamma)
    for r in range(w.n_replicas):
        for x, y in zip(a.export(r), b.export(r)):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("path", ["auto", "streamed"])
def test_batch_dd_and_ghz_circuits_with_pulses(B, orc, path):
    """A small batch shaped like the batched configuration (DD circuits with their own ideal
    pulses, GHZ circuits, uneven n and walker targets): every circuit equals its oracle."""
    bw = W.batch(n_circuits=10, n_lo=3, n_hi=6, n_replicas=2, nsteps=600, w_lo=1e3, w_hi=2e4,
                 seed=7)
    R = bw.n_replicas
    circuits = [(w.h, w.lops, w.init_keys, w.init_re, w.init_im) for w in bw.circuits]
    _say(f"{bw.name}: n={bw.n}, {len(circuits)} circuits, {path}")
    g = B.QMC.batch(bw.n, R, bw.seed, bw.dt, circuits, store_capacity=1 << 14,
                    spawn_capacity=1 << 16)
    g.set_path(path)
    orcs = _oracles(orc, bw.n, R, bw.seed, bw.dt, circuits)
    for a, b, masks in bw.segments():
        if masks is not None:
            g.pulse_batch(*masks)
            for c, o in enumerate(orcs):
                if masks[0][c] or masks[1][c]:
                    o.pulse(int(masks[0][c]), int(masks[1][c]))
        s, gam = bw.weights(a, b)
        g.step(s, gam)
        for c, (o, w) in enumerate(zip(orcs, bw.circuits)):
            o.step(w.s[a:b], w.gamma[a:b])
    _same(g, orcs, R, f"step {bw.nsteps}")


def test_batch_refuses_ab2_and_initiator(B):
    rng = np.random.default_rng(3)
    circuits = []
    for c in range(2):
        h, lops = W.random_model(3, rng, n_h=3, n_l=1)
        circuits.append((h, lops, [0], [100], [0]))
    g = B.QMC.batch(3, 2, 1, 0.01, circuits, store_capacity=64, spawn_capacity=1024)
    with pytest.raises(B.QMCError) as e:
        g.set_integrator("ab2")
    assert e.value.code == B.QMC_ERR_ARG
    with pytest.raises(B.QMCError) as e:
        g.set_initiator(10)
    assert e.value.code == B.QMC_ERR_ARG


def test_batch64_full_size_sampled_circuits(B, orc):
    """The batched configuration at full size (64 circuits, 1000 steps, automatic path, sort tile
    autotuned: the launch configuration of the benchmark): the four circuits with the smallest
    walker targets, whose oracles finish in seconds, equal their oracles at steps 500 and 1000;
    every other circuit's store is checked to be sorted, unique and free of empty records."""
    bw = W.config_batch64()
    R = bw.n_replicas
    circuits = [(w.h, w.lops, w.init_keys, w.init_re, w.init_im) for w in bw.circuits]
    _say(f"{bw.name}: n={bw.n}, {len(circuits)} circuits, {bw.nsteps} steps, automatic path")
    g = B.QMC.batch(bw.n, R, bw.seed, bw.dt, circuits, store_capacity=1 << 18,
                    spawn_capacity=1 << 18)
    g.tune_sort(0)
    pick = sorted(range(len(bw.circuits)),
                  key=lambda c: (bw.circuits[c].walker_target, bw.circuits[c].n))[:4]
    orcs = {}
    for c in pick:
        h, lops, keys, re, im = circuits[c]
        o = orc.Oracle(bw.n, R, bw.seed, bw.dt, h, lops, keys, re, im)
        o.set_replica_base(c * R)
        orcs[c] = o
    checkpoints = {500, bw.nsteps}
    for a, b, masks in bw.segments():
        cuts = sorted({a, b} | {x for x in checkpoints if a < x < b})
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            if lo == a and masks is not None:
                g.pulse_batch(*masks)
                for c, o in orcs.items():
                    if masks[0][c] or masks[1][c]:
                        o.pulse(int(masks[0][c]), int(masks[1][c]))
            s, gam = bw.weights(lo, hi)
            g.step(s, gam)
            for c, o in orcs.items():
                o.step(bw.circuits[c].s[lo:hi], bw.circuits[c].gamma[lo:hi])
            if hi in checkpoints:
                for c, o in orcs.items():
                    for r in range(R):
                        for x, y in zip(g.export(c * R + r), o.export(r)):
                            assert np.array_equal(x, y), f"step {hi}: circuit {c} replica {r}"
                _say(f"  step {hi}: circuits {pick} equal their oracles")
    for seg in range(len(circuits) * R):
        k, a, b = g.export(seg)
        assert np.all(np.diff(k.astype(np.int64)) > 0) if len(k) > 1 else True
        assert not np.any((a == 0) & (b == 0))
