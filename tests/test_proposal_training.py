"""Host-side helpers of the proposal trainer (paper_2502_18929_amd.proposal): spawn events pooled
per parent key against a count event by event, and the quantized network's integer scores
against the oracle's MLP scores."""
import numpy as np
import pytest

from paper_2502_18929_amd import binding, proposal as PR, workloads as W

_EV = np.dtype([("key", "<u8"), ("step", "<u4"), ("group", "<u4"), ("re", "<i4"), ("im", "<i4")])


@pytest.fixture(scope="module")
def lib_built():
    import os
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libqmc.so not built")
    binding.lib()


def test_pooled_fractions_by_brute_force():
    """Spawn events pooled per parent key: walkers per column group over the key's total,
    counted here event by event; groups past N_OUT and the diagonal are left out."""
    rng = np.random.default_rng(1700)
    n = 5
    m = 4000
    ev = np.zeros(m, dtype=_EV)
    ev["key"] = (rng.integers(0, 40, size=m).astype(np.uint64) |
                 (rng.integers(0, 4, size=m).astype(np.uint64) << np.uint64(2 * n)))
    ev["step"] = rng.integers(0, 100, size=m)
    ev["group"] = rng.integers(0, PR.N_OUT + 3, size=m)
    ev["re"] = rng.integers(-5, 6, size=m)
    ev["im"] = rng.integers(-5, 6, size=m)
    keys, Y, tot, nev = PR.pooled_fractions(ev, n)
    want, cnt = {}, {}
    for e in ev:
        g = int(e["group"])
        if 1 <= g <= PR.N_OUT:
            k = int(e["key"]) & ((1 << (2 * n)) - 1)
            want.setdefault(k, np.zeros(PR.N_OUT))[g - 1] += abs(int(e["re"])) + abs(int(e["im"]))
            cnt[k] = cnt.get(k, 0) + 1
    assert sorted(want) == [int(k) for k in keys]
    for i, k in enumerate(keys):
        row = want[int(k)]
        assert tot[i] == row.sum() and nev[i] == cnt[int(k)]
        assert np.allclose(Y[i], row / max(row.sum(), 1))


def test_quantized_scores_are_the_oracle_network(orc, lib_built):
    rng = np.random.default_rng(1710)
    n = 6
    keys = np.unique(rng.integers(0, 1 << (2 * n), size=3000).astype(np.uint64))
    tgt = rng.random((len(keys), PR.N_OUT)) * (keys[:, None] % 7 + 1).astype(np.float64)
    params = PR.fit(keys, tgt, 2 * n, iters=50)
    mlp = PR.quantize(params, keys, 2 * n)
    assert mlp[0].dtype == np.int8 and mlp[0].shape == (32, 64)
    assert mlp[2].dtype == np.int8 and mlp[2].shape == (64, 32)
    assert 0 <= mlp[4] <= 30
    o = orc.Oracle(n, 1, 1, 0.01, [], [], keys[:1], np.ones(1, np.int32), np.zeros(1, np.int32))
    o.set_proposal("mlp", 1, mlp)
    sc = PR.scores(mlp, keys[:200], 2 * n)
    for i, key in enumerate(keys[:200]):
        assert np.array_equal(sc[i], o.mlp_scores(int(key)))


# ---- the deeper network's trainer ------------------------------------------------------------



def test_deep_features_are_key_signs_then_channel_bits():
    keys = np.array([0b1011, 0], dtype=np.uint64)
    x = PR.deep_features(keys, [0b101, (1 << 124) | (1 << 90) | 1], 4)
    assert x.shape == (2, 128)
    assert x[0, :4].tolist() == [1, 1, -1, 1] and x[0, 4:8].tolist() == [1, 0, 1, 0]
    assert x[1, :4].tolist() == [-1, -1, -1, -1] and x[1, 4] == 1 and x[1, 4 + 90] == 1
    assert x[1, 4:].sum() == 2   # channel 124 would be input 128: past the network's inputs
    assert x[0, 8:].sum() == 0


def test_deep_training_set_sums_walkers_per_key_window_and_group():
    """Two windows of a workload (the channel masks of its steps): events of one parent key in the
    same window pool, groups split, fractions sum to one, the weight is the walker total."""
    w = W.config_ghz4()
    masks = PR.active_masks(w)
    a = next(k for k in range(w.nsteps) if masks[k] != masks[0])   # first step of window two
    ev = np.zeros(5, dtype=_EV)
    ev["key"] = [7, 7 | (1 << 8), 7, 7, 3]        # the second carries a segment tag
    ev["step"] = [0, 1, 2, a, 0]
    ev["group"] = [1, 2, 1, 1, 3]
    ev["re"] = [2, -1, 0, 5, 1]
    ev["im"] = [0, 0, -3, 0, 0]
    keys, pm, Y, tot = PR.deep_training_set(ev, w)
    got = {(int(k), m): (y, t) for k, m, y, t in zip(keys, pm, Y, tot)}
    y, t = got[(7, masks[0])]
    assert t == 6 and y[0] == pytest.approx(5 / 6) and y[1] == pytest.approx(1 / 6)
    y, t = got[(7, masks[a])]
    assert t == 5 and y[0] == 1
    assert got[(3, masks[0])][0][2] == 1
    assert len(got) == 3


def test_proposal_variance_factor():
    """sum_g t_g^2 / q_g under the kernel's thresholds: G - 1 for a one-hot target under uniform
    weights, close to 1 when the weights are the fractions (the floor keeps it above)."""
    Y = np.zeros((3, PR.DEEP_OUT))
    Y[0, 2] = 1
    Y[1, :4] = 0.25
    Y[2, 0], Y[2, 5] = 0.9, 0.1
    G = np.array([11, 5, 8])
    uni = PR.proposal_variance(np.ones((3, PR.DEEP_OUT)), Y, G)
    assert uni == pytest.approx((10 + 1 + (0.81 + 0.01) * 7) / 3)
    exact = PR.proposal_variance(np.rint(Y * 2 ** 20), Y, G)
    assert 1.0 <= exact < 1.1
    zero = PR.proposal_variance(np.zeros((3, PR.DEEP_OUT)), Y, G)
    assert zero == pytest.approx(uni)   # all-zero weights are the uniform proposal


def test_deep_quantized_scores_are_the_oracle_network(orc):
    rng = np.random.default_rng(1720)
    n = 5
    keys = np.unique(rng.integers(0, 1 << (2 * n), size=2000).astype(np.uint64))
    masks = [int(m) for m in rng.integers(0, 1 << 40, size=len(keys))]
    X = PR.deep_features(keys, masks, 2 * n)
    Y = rng.random((len(keys), PR.DEEP_OUT))
    Y /= Y.sum(axis=1, keepdims=True)
    G = np.full(len(keys), 20)
    params = PR.fit_deep(X, Y, np.ones(len(keys)), G, iters=30)
    net = PR.quantize_deep(params, X)
    assert net[0].dtype == np.int8 and net[2].dtype == np.int8 and net[4].dtype == np.int8
    assert 0 <= net[6] <= 30 and 0 <= net[7] <= 30
    o = orc.Oracle(n, 1, 1, 0.01, [], [], keys[:1], np.ones(1, np.int32), np.zeros(1, np.int32))
    o.set_proposal_deep(1, net)
    sc = PR.deep_scores(net, X[:100])
    for i in range(100):
        assert np.array_equal(sc[i], o.deep_scores(int(keys[i]), masks[i]))
