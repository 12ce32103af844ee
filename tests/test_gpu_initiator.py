"""GPU parity of the initiator approximation (End Matter on simulation methodology, reading R17)
against the oracle: whole per-replica stores compared bit for bit, on both step paths, with the
Euler and the AB2 integrator.  Both sides run their own trajectories from the same records."""
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


def _same(g, o, R, where):
    for r in range(R):
        for a, b in zip(g.export(r), o.export(r)):
            if not np.array_equal(a, b):
                raise AssertionError(f"{where} replica {r}: sizes {len(g.export(r)[0])} / "
                                     f"{len(o.export(r)[0])}")


@pytest.mark.parametrize("integ", ["euler", "ab2"])
@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(3))
def test_initiator_random_models_every_step(B, orc, seed, path, integ):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(2, 5))
    h, lops = W.random_model(n, rng, n_h=int(rng.integers(2, 7)), n_l=int(rng.integers(1, 4)))
    keys, re, im = W.random_records(n, rng, int(rng.integers(2, 10)), scale=400)
    R = int(rng.integers(1, 5))
    T = int(rng.integers(50, 400))
    _say(f"initiator seed={seed} n={n} R={R} T={T} path={path} {integ}")
    g = B.QMC(n, R, 77 + seed, 0.01, h, lops, keys, re, im, store_capacity=1 << (2 * n),
              spawn_capacity=1 << 14)
    g.set_path(path)
    g.set_integrator(integ)
    g.set_initiator(T)
    o = orc.Oracle(n, R, 77 + seed, 0.01, h, lops, keys, re, im, integrator=integ)
    o.set_initiator(T)
    s = rng.normal(size=(40, len(h)))
    gam = np.abs(rng.normal(size=(40, len(lops))))
    for k in range(40):
        g.step(s[k:k + 1], gam[k:k + 1])
        o.step(s[k:k + 1], gam[k:k + 1])
        _same(g, o, R, f"step {k}")


@pytest.mark.parametrize("path", PATHS)
def test_initiator_off_again_is_the_plain_step(B, orc, path):
    """Threshold on for 60 steps, then 0: the oracle does the same switch."""
    w = W.config_ghz4()
    T = B.initiator_threshold("0.01", w.walker_target)
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=8192)
    g.set_path(path)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    g.set_initiator(T)
    o.set_initiator(T)
    g.step(w.s[:60], w.gamma[:60])
    o.step(w.s[:60], w.gamma[:60])
    _same(g, o, w.n_replicas, "step 60")
    g.set_initiator(0)
    o.set_initiator(0)
    g.step(w.s[60:200], w.gamma[60:200])
    o.step(w.s[60:200], w.gamma[60:200])
    _same(g, o, w.n_replicas, "step 200")


@pytest.mark.parametrize("integ", ["euler", "ab2"])
@pytest.mark.parametrize("path", ["auto", "streamed"])
def test_initiator_ghz20_nm_full_size(B, orc, path, integ):
    """n=20 non-Markovian GHZ at full size with xi = 0.1 % (the paper's setting): all 3000
    steps, every replica compared every 500 steps."""
    w = W.config_ghz20_nm()
    T = B.initiator_threshold("0.001", w.walker_target)
    _say(f"initiator {w.name}: T={T}, {path}, {integ}")
    g = B.QMC.from_workload(w, store_capacity=1 << 17, spawn_capacity=1 << 20)
    g.set_path(path)
    g.set_integrator(integ)
    g.set_initiator(T)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im, integrator=integ)
    o.set_initiator(T)
    for k0 in range(0, w.nsteps, 500):
        g.step(w.s[k0:k0 + 500], w.gamma[k0:k0 + 500])
        o.step(w.s[k0:k0 + 500], w.gamma[k0:k0 + 500], threads=16)
        _same(g, o, w.n_replicas, f"step {k0 + 500}")
        _say(f"  step {k0 + 500} equal, {g.counters()['n_occ']} keys")


@pytest.mark.parametrize("path", PATHS)
def test_initiator_dd12_first_steps(B, orc, path):
    """n=12 DD with crosstalk (16 replicas x 1e6 walkers, pulses included), xi = 0.1 %, first
    400 steps."""
    w = W.config_dd12()
    T = B.initiator_threshold("0.001", w.walker_target)
    _say(f"initiator {w.name}: T={T}, {path}")
    g = B.QMC.from_workload(w, store_capacity=1 << 20, spawn_capacity=1 << 21)
    g.set_path(path)
    g.set_initiator(T)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    o.set_initiator(T)
    for a, b, pulses in w.segments():
        if a >= 400:
            break
        for (px, pz) in pulses:
            g.pulse(px, pz)
            o.pulse(px, pz)
        b = min(b, 400)
        g.step(w.s[a:b], w.gamma[a:b])
        o.step(w.s[a:b], w.gamma[a:b], threads=16)
    _same(g, o, w.n_replicas, "step 400")


def test_initiator_needs_a_free_key_bit(B):
    """2n + replica bits = 63 leaves one bit: accepted; 64 leaves none: refused."""
    h = [(1, 0, 0.5)]
    ok = B.QMC(31, 2, 1, 0.01, h, [], [0], [10], [0], store_capacity=4, spawn_capacity=16)
    ok.set_initiator(5)
    full = B.QMC(31, 4, 1, 0.01, h, [], [0], [10], [0], store_capacity=4, spawn_capacity=16)
    with pytest.raises(B.QMCError) as e:
        full.set_initiator(5)
    assert e.value.code == B.QMC_ERR_ARG
    full.set_initiator(0)
