"""GPU parity of the variable shift (population control of the FCIQMC background paragraph,
update rule of Booth et al. 2009; off by default): both step paths against the oracle, whole
stores bit for bit and the shifts themselves exactly, since both sides compute the same FP64
update from the same integer N^tot."""
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


@pytest.mark.parametrize("path", ["fused", "streamed"])
@pytest.mark.parametrize("seed", range(3))
def test_variable_shift_random_models(B, orc, seed, path):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(2, 5))
    h, lops = W.random_model(n, rng, n_h=int(rng.integers(1, 5)), n_l=int(rng.integers(1, 3)))
    keys, re, im = W.random_records(n, rng, 6, scale=400)
    R, dt, A = 3, 0.01, int(rng.integers(2, 7))
    nt0 = int(np.abs(re).sum() + np.abs(im).sum())
    ctl = {"zeta": 0.25, "period": A, "target": int(nt0 * 1.05)}
    g = B.QMC(n, R, 31 + seed, dt, h, lops, keys, re, im, store_capacity=1 << 12,
              spawn_capacity=1 << 14, shift=ctl)
    g.set_path(path)
    o = orc.Oracle(n, R, 31 + seed, dt, h, lops, keys, re, im)
    o.set_shift_control(1, ctl["zeta"], A, ctl["target"])
    for r in range(R):          # a growing start so that the replicas reach the target
        g.set_shift(r, 1.5 + 0.5 * r)
        o.set_shift(r, 1.5 + 0.5 * r)
    s = rng.uniform(-1, 1, size=(1, len(h)))
    gam = rng.uniform(0.05, 0.5, size=(1, len(lops)))
    for chunk in (7, 13, 40):   # calls that do not end on period boundaries
        g.step(np.repeat(s, chunk, 0), np.repeat(gam, chunk, 0))
        o.step(np.repeat(s, chunk, 0), np.repeat(gam, chunk, 0))
        _same(g, o, R, f"{path} seed {seed}")
        got = g.observe()
        for r in range(R):
            assert got["shift"][r] == o.shift(r)
    assert any(o.shift(r) != 1.5 + 0.5 * r for r in range(R))   # the control acted
    assert got["biased"]


@pytest.mark.parametrize("path", ["fused", "streamed"])
def test_variable_shift_ghz4(B, orc, path):
    w = W.config_ghz4()
    ctl = {"zeta": 0.1, "period": 10, "target": 10500}
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096, shift=ctl)
    g.set_path(path)
    o = orc.Oracle(w.n, w.n_replicas, w.seed, w.dt, w.h, w.lops, w.init_keys, w.init_re,
                   w.init_im)
    o.set_shift_control(1, ctl["zeta"], ctl["period"], ctl["target"])
    for r in range(w.n_replicas):
        g.set_shift(r, 0.3)
        o.set_shift(r, 0.3)
    for a in range(0, w.nsteps, 100):
        g.step(w.s[a:a + 100], w.gamma[a:a + 100])
        o.step(w.s[a:a + 100], w.gamma[a:a + 100])
        _same(g, o, w.n_replicas, f"step {a + 100}")
    got = g.observe()
    assert [got["shift"][r] for r in range(w.n_replicas)] == \
        [o.shift(r) for r in range(w.n_replicas)]


def test_variable_shift_batch(B, orc):
    """Two circuits of a batch: every segment (circuit, replica) has its own shift and N^tot."""
    rng = np.random.default_rng(77)
    circuits = []
    for c in range(2):
        h, lops = W.random_model(3, rng, n_h=3, n_l=1)
        keys, re, im = W.random_records(3, rng, 4, scale=300)
        circuits.append((h, lops, keys, re, im))
    R, A = 2, 4
    ctl = {"zeta": 0.3, "period": A, "target": 0}
    g = B.QMC.batch(3, R, 9, 0.01, circuits, store_capacity=512, spawn_capacity=4096,
                    shift=ctl)
    orcs = []
    for c, (h, lops, keys, re, im) in enumerate(circuits):
        o = orc.Oracle(3, R, 9, 0.01, h, lops, keys, re, im)
        o.set_replica_base(c * R)
        o.set_shift_control(1, ctl["zeta"], A, 0)
        orcs.append(o)
    s = [rng.uniform(-1, 1, size=(30, len(c[0]))) for c in circuits]
    gam = [rng.uniform(0.05, 0.4, size=(30, len(c[1]))) for c in circuits]
    g.step(np.concatenate(s, axis=1), np.concatenate(gam, axis=1))
    for c, o in enumerate(orcs):
        o.step(s[c], gam[c])
        for r in range(R):
            for x, y in zip(g.export(c * R + r), o.export(r)):
                assert np.array_equal(x, y), (c, r)
    got = g.observe()
    for c, o in enumerate(orcs):
        for r in range(R):
            assert got["shift"][c * R + r] == o.shift(r)


def test_variable_shift_refusals(B):
    w = W.config_ghz4()
    with pytest.raises(B.QMCError) as e:
        B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096,
                            shift={"zeta": 0.1, "period": 0})
    assert e.value.code == B.QMC_ERR_ARG
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096,
                            shift={"zeta": 0.1, "period": 5})
    with pytest.raises(B.QMCError) as e:
        g.set_integrator("ab2")
    assert e.value.code == B.QMC_ERR_ARG
