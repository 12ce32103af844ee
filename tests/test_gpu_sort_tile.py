"""The sort-tile autotuner of the streamed path (qmc_tune_sort): every tile size gives the
oracle's walkers bit for bit, tuning leaves the state alone, and unsupported sizes are
refused."""
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


def _same(g, o, R):
    for r in range(R):
        for a, b in zip(g.export(r), o.export(r)):
            assert np.array_equal(a, b), f"replica {r}"


def _case():
    rng = np.random.default_rng(1800)
    n, R = 7, 2
    h, lops = W.random_model(n, rng, n_h=8, n_l=3)
    keys = np.arange(1 << (2 * n), dtype=np.uint64)[::2]
    re = rng.integers(-60, 60, size=len(keys)).astype(np.int32)
    im = rng.integers(-60, 60, size=len(keys)).astype(np.int32)
    re[(re == 0) & (im == 0)] = 5
    s = rng.normal(size=(4, len(h))) * 0.4
    gam = np.abs(rng.normal(size=(4, len(lops)))) * 0.4
    return n, R, h, lops, keys, re, im, s, gam


@pytest.mark.parametrize("ipt", [8, 12, 16, 24])
def test_every_tile_size_matches_the_oracle(B, orc, ipt):
    n, R, h, lops, keys, re, im, s, gam = _case()
    _say(f"sort tile {ipt} records/thread: {len(keys)} keys x {R} replicas, streamed")
    g = B.QMC(n, R, 4, 0.01, h, lops, keys, re, im, store_capacity=1 << 15,
              spawn_capacity=1 << 20)
    g.set_path("streamed")
    assert g.tune_sort(ipt) == ipt
    o = orc.Oracle(n, R, 4, 0.01, h, lops, keys, re, im)
    g.step(s, gam)
    o.step(s, gam, threads=2)
    _same(g, o, R)


def test_autotune_keeps_the_state_and_the_results(B, orc):
    n, R, h, lops, keys, re, im, s, gam = _case()
    g = B.QMC(n, R, 4, 0.01, h, lops, keys, re, im, store_capacity=1 << 15,
              spawn_capacity=1 << 20)
    g.set_path("streamed")
    o = orc.Oracle(n, R, 4, 0.01, h, lops, keys, re, im)
    g.step(s[:2], gam[:2])
    o.step(s[:2], gam[:2], threads=2)
    before = [g.export(r) for r in range(R)]
    chosen = g.tune_sort()
    _say(f"autotuned sort tile: {chosen} records/thread")
    assert chosen in (8, 12, 16, 24)
    for r in range(R):
        for a, b in zip(before[r], g.export(r)):
            assert np.array_equal(a, b)
    g.step(s[2:], gam[2:])
    o.step(s[2:], gam[2:], threads=2)
    _same(g, o, R)


def test_unsupported_tile_is_refused(B):
    g = B.QMC(1, 1, 1, 0.01, [], [], [0], [1], [0], store_capacity=4, spawn_capacity=4)
    for bad in (1, 10, 32):
        with pytest.raises(B.QMCError) as e:
            g.tune_sort(bad)
        assert e.value.code == B.QMC_ERR_ARG
