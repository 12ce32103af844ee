"""Host-side helpers of the proposal trainer (paper_2502_18929_amd.proposal) against the oracle:
the per-group coefficient magnitudes are the oracle's quantized column entries, and the
quantized network's integer scores are the oracle's MLP scores."""
import numpy as np
import pytest

from paper_2502_18929_amd import binding, proposal as PR, workloads as W


@pytest.fixture(scope="module")
def lib_built():
    import os
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libqmc.so not built")
    binding.lib()


@pytest.mark.parametrize("seed", range(3))
def test_group_magnitudes_are_the_column_entries(orc, lib_built, seed):
    rng = np.random.default_rng(1700 + seed)
    n = 3
    h, lops = W.random_model(n, rng, n_h=5, n_l=3)
    s = rng.normal(size=len(h))
    gam = np.abs(rng.normal(size=len(lops)))
    tab = binding.coeff_table(n, 0.01, h, lops, s, gam)
    keys = np.arange(1 << (2 * n), dtype=np.uint64)
    m = PR.group_magnitudes(tab, keys)
    o = orc.Oracle(n, 1, 1, 0.01, h, lops, keys[:1], np.ones(1, np.int32), np.zeros(1, np.int32))
    for key in keys[::5]:
        tk, v = o.column_q(s, gam, int(key))
        col = {int(t): abs(int(a)) + abs(int(b)) for t, (a, b) in zip(tk, v)}
        for g in range(1, len(tab["gxmask"])):
            want = col.get(int(key) ^ int(tab["gxmask"][g]), 0)
            assert m[int(key), g - 1] == want


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
