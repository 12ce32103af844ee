"""CPU-only checks of the HIP library's host side: the shared library loads and exports every
symbol include/qmc.h declares, and its per-step coefficient table (quantization, merging,
grouping, bound check) equals the oracle's bit for bit.  No device calls."""
import os
import re

import numpy as np
import pytest

from paper_2502_18929_amd import binding, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qmc.h")).read()
    return sorted(set(re.findall(r"\b(qmc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    names = _declared()
    assert "qmc_init" in names and "qmc_step" in names and "qmc_observe" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(binding.EXPORTED) == names


def _tables_equal(a, b):
    for k in ("gxmask", "gstart", "zmask", "q"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("scale", [1.0, 1.5, -0.5])
@pytest.mark.parametrize("cfg", ["ghz4", "dd12", "ghz20_nm"])
def test_coeff_tables_match_oracle_on_configs(orc, cfg, scale):
    """Euler tables (scale 1) and the two AB2 tables (3/2, -1/2), bit for bit."""
    w = W.CONFIGS[cfg]()
    o = orc.Oracle(w.n, 1, 1, w.dt, w.h, w.lops, w.init_keys, w.init_re, w.init_im)
    idx = sorted(set([0, 1, w.nsteps // 3, w.nsteps // 2, w.nsteps - 1] +
                     list(range(0, w.nsteps, max(1, w.nsteps // 25)))))
    for k in idx:
        a = binding.coeff_table(w.n, w.dt, w.h, w.lops, w.s[k], w.gamma[k], scale=scale)
        b = o.table(w.s[k], w.gamma[k], scale=scale)
        _tables_equal(a, b)


@pytest.mark.parametrize("seed", range(8))
def test_coeff_tables_match_oracle_random(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 7))
    h, lops = W.random_model(n, rng, n_h=int(rng.integers(0, 8)), n_l=int(rng.integers(0, 4)),
                             max_l_terms=3)
    dt = float(rng.choice([0.001, 0.01, 0.02]))
    s = rng.normal(size=len(h))
    g = rng.normal(size=len(lops))
    o = orc.Oracle(n, 1, 1, dt, h, lops, [0], [1], [0])
    try:
        b = o.table(s, g)
    except orc.OracleError as e:
        with pytest.raises(binding.QMCError) as e2:
            binding.coeff_table(n, dt, h, lops, s, g)
        assert e2.value.code == e.code
        return
    a = binding.coeff_table(n, dt, h, lops, s, g)
    _tables_equal(a, b)


def test_quantization_ties_round_half_even(orc):
    """Coefficients landing exactly halfway between Q32 steps round half to even, both below
    2^51 and above it (a pair of huge terms on one mask whose rounded sum is small)."""
    n = 3
    dt = 2.0 ** -33  # dt * c * 2^32 = c / 2: odd integers c give exact ties
    h = [(x, z, float(2 * (4 * x + z) + 1) * (-1) ** z) for x in range(1, 4) for z in range(4)]
    h += [(0, 1, 2.0 ** 52 + 1), (0, 1, -(2.0 ** 52 + 3)), (0, 2, 2.0 ** 53 + 2.0),
          (0, 2, -(2.0 ** 53) - 6.0)]
    s = np.ones(len(h))
    o = orc.Oracle(n, 1, 1, dt, h, [], [0], [1], [0])
    b = o.table(s, np.zeros(0))
    a = binding.coeff_table(n, dt, h, [], s, np.zeros(0))
    _tables_equal(a, b)
    d0, d1 = int(a["gstart"][0]), int(a["gstart"][1])  # the diagonal group
    q = dict(zip(a["zmask"][d0:d1].tolist(), a["q"][d0:d1].tolist()))
    # -i h gives Im = -Re(h): ties -(2^51 + 1/2) -> -2^51, 2^51 + 3/2 -> 2^51 + 2, and above
    # 2^52 (spacing 1) the halves -(2^52 + 1) and 2^52 + 3 are already integers
    assert q[1][1] == -(2 ** 51) + (2 ** 51 + 2)
    assert q[2][1] == -(2 ** 52 + 1) + (2 ** 52 + 3)


def test_dt_bound_rejected_like_oracle(orc):
    w = W.config_ghz4()
    with pytest.raises(binding.QMCError) as e:
        binding.coeff_table(w.n, 0.5, w.h, w.lops, w.s[0] * 10, w.gamma[0])
    assert e.value.code == binding.QMC_ERR_DT
    o = orc.Oracle(w.n, 1, 1, 0.5, w.h, w.lops, w.init_keys, w.init_re, w.init_im)
    with pytest.raises(orc.OracleError) as e2:
        o.table(w.s[0] * 10, w.gamma[0])
    assert e2.value.code == orc.ORC_ERR_DT


def test_invalid_configuration_rejected():
    with pytest.raises(binding.QMCError):
        binding.coeff_table(33, 0.01, [], [], [], [])
    with pytest.raises(binding.QMCError):
        binding.coeff_table(2, 0.01, [(4, 0, 1.0)], [], [1.0], [])   # mask outside n bits


def test_initiator_threshold_rounds_up_exactly():
    """ceil(xi * N^diag) in exact rational arithmetic (0.001 * 1e7 is 10000, not 10001)."""
    assert binding.initiator_threshold("0.001", 10_000_000) == 10_000
    assert binding.initiator_threshold(0.001, 1_000_000) == 1_000
    assert binding.initiator_threshold("0.001", 10_001) == 11
    assert binding.initiator_threshold("0.1", 3) == 1
    assert binding.initiator_threshold(0, 10 ** 9) == 0
