"""Host-side pieces of the benchmark: the error bar behind the time-to-error-bar half of the
metric, a 95 % bootstrap confidence interval over the replicas (the paper's error bars, End Matter
on simulation methodology)."""
import numpy as np
import pytest

import bench


class _W:
    def __init__(self, labels):
        self.pauli_obs = [(lab, 0, 1, 1.0) for lab in labels]


def _obs(fid, pauli):
    R = len(fid)
    pv = np.zeros((R, pauli.shape[1], 2))
    pv[:, :, 0] = pauli
    return {"fidelity": np.stack([fid, np.zeros(R)], axis=1), "pauli_val": pv}


def test_error_bar_matches_normal_interval():
    # for many replicas the bootstrap percentile interval of the mean approaches the normal one,
    # 1.96 sigma / sqrt(R)
    rng = np.random.default_rng(5)
    R, sig = 400, 0.1
    fid = 0.5 + sig * rng.standard_normal(R)
    eb = bench.error_bar(_obs(fid, np.zeros((R, 1))), _W(["Z0"]), 2.0)
    ref = 1.96 * fid.std(ddof=1) / np.sqrt(R)
    assert eb["ci95_halfwidth_fidelity"] == pytest.approx(ref, rel=0.1)
    assert eb["widest"] == "fidelity" and eb["ci95_halfwidth_max"] == eb["ci95_halfwidth_fidelity"]
    assert eb["reached"] and eb["wall_s"] == 2.0


def test_error_bar_widest_observable_and_extrapolation():
    rng = np.random.default_rng(6)
    R = 16
    fid = np.full(R, 0.7)                      # no spread: zero width
    pauli = np.stack([0.01 * rng.standard_normal(R), 0.4 * rng.standard_normal(R)], axis=1)
    eb = bench.error_bar(_obs(fid, pauli), _W(["Z0", "Z1"]), 3.0)
    assert eb["ci95_halfwidth_fidelity"] == 0.0
    assert eb["widest"] == "Z1"
    h = eb["ci95_halfwidth_max"]
    assert h > bench.ERROR_BAR and not eb["reached"]
    assert eb["wall_s"] == pytest.approx(3.0 * (h / bench.ERROR_BAR) ** 2)


def test_error_bar_needs_two_replicas():
    assert bench.error_bar(_obs(np.array([0.5]), np.zeros((1, 1))), _W(["Z0"]), 1.0) is None
