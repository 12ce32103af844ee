"""Streamed chunks captured as HIP graphs (qmc_use_graphs): every replay, with eager calls in
between, gives the oracle's walkers bit for bit."""
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
        for a, b in zip(g.export(r), o.export(r)):
            assert np.array_equal(a, b), f"{where}: replica {r}"


@pytest.mark.parametrize("integrator", ["euler", "ab2"])
def test_graph_replays_match_the_oracle(B, orc, integrator):
    rng = np.random.default_rng(1900)
    n, R = 5, 3
    h, lops = W.random_model(n, rng, n_h=6, n_l=3)
    keys, re, im = W.random_records(n, rng, 200, scale=2000)
    steps = 40
    s = rng.normal(size=(steps, len(h))) * 0.4
    gam = np.abs(rng.normal(size=(steps, len(lops)))) * 0.4
    g = B.QMC(n, R, 6, 0.01, h, lops, keys, re, im, store_capacity=1 << 10,
              spawn_capacity=1 << 16)
    g.set_path("streamed")
    g.set_integrator(integrator)
    o = orc.Oracle(n, R, 6, 0.01, h, lops, keys, re, im, integrator=integrator)
    # calls of 5 steps (the same launches: the executable graph is updated and replayed), one of
    # 3 (new launches: a new graph), and eager calls in between
    k = 0
    for size, graph in [(5, True), (5, True), (5, True), (3, True), (5, False), (5, True),
                        (2, False), (5, True), (5, True)]:
        g.use_graphs(graph)
        g.step(s[k:k + size], gam[k:k + size])
        o.step(s[k:k + size], gam[k:k + size])
        k += size
        _same(g, o, R, f"after step {k} ({'graph' if graph else 'eager'})")
    _say(f"{integrator}: {k} steps in graph and eager calls, all equal")


def test_graph_dd_with_pulses(B, orc):
    w = W.dd(n=6, n_replicas=4, walker_target=20000, nsteps=800, seed=11)
    g = B.QMC.from_workload(w, store_capacity=4096, spawn_capacity=1 << 16)
    g.set_path("streamed")
    g.use_graphs(True)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    stop = min(w.nsteps, 400)
    for a, b, pulses in w.segments():
        if a >= stop:
            break
        for (px, pz) in pulses:
            g.pulse(px, pz)
            o.pulse(px, pz)
        g.step(w.s[a:min(b, stop)], w.gamma[a:min(b, stop)])
        o.step(w.s[a:min(b, stop)], w.gamma[a:min(b, stop)], threads=4)
    _same(g, o, w.n_replicas, f"DD after {stop} steps")
