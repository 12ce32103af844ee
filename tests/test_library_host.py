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
