"""Host-side pieces of the benchmark: the error bar behind the time-to-error-bar half of the
metric, a 95 % bootstrap confidence interval over the replicas (the paper's error bars, End Matter
on simulation methodology), and the roofline object (the per-step algorithmic bytes, the timed
class and the class reported beside it)."""
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


# ---- the roofline object: algorithmic bytes of the per-step unit ---------------------------------

_COV = dict(steps=100, walker_steps=10 ** 9, key_steps=4_000_000, child_steps=300_000,
            out_steps=4_100_000, spawn_steps=250_000)


def test_step_bytes_are_the_per_step_formula():
    # 16 B per record: read to spawn, diagonal write-back (8 B), children written and read, read to
    # annihilate, survivors written
    want = 16 * 4_000_000 + 8 * 4_000_000 + 2 * 16 * 250_000 + 16 * 4_000_000 + 16 * 4_100_000
    assert bench.step_bytes(_COV) == want
    for kind in ("fused", "small", "step"):
        assert bench.algorithmic_bytes(kind, _COV) == want
    assert bench.algorithmic_bytes("merge", _COV) == 16 * (4_000_000 + 250_000 + 4_100_000)


def test_roofline_of_a_timed_class():
    r = bench.roofline("step", "no_such_workload", 20.0, 4, _COV)
    per = bench.step_bytes(_COV) / 4
    assert r["algorithmic_bytes_per_launch"] == per
    assert r["avg_launch_ms"] == 5.0 and r["steps_per_launch"] == 25.0
    assert r["achieved"] == pytest.approx(per / 5e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
    assert r["kernel_us_per_step"] == pytest.approx(200.0)
    assert r["kernel"] == "streamed_step" and r["traffic"] is None  # no committed summary
    empty = bench.roofline("small", "no_such_workload", 0.0, 0, dict(_COV, steps=0))
    assert empty["achieved"] == 0.0 and empty["kernel_us_per_step"] is None


class _Ctx:
    """Stands in for a context's profile totals: (ms, launches, covered) per class."""
    def __init__(self, totals):
        self.totals = totals

    def profile_read(self, kind=None):
        return self.totals[kind]


def test_whole_step_class_reports_the_longer_whole_step_kernel():
    cov_f, cov_s = dict(_COV, steps=1800), dict(_COV, steps=1200)
    g = _Ctx({"fused": (39.0, 1, cov_f), "small": (10.8, 48, cov_s)})
    kind, ms, n, cov, other = bench.whole_step_class(g, "small")
    assert kind == "fused" and ms == 39.0 and n == 1 and cov["steps"] == 1800
    assert other == {"kernel": "k_small", "ms": 10.8, "launches": 48, "steps_covered": 1200}


def test_whole_streamed_step_carries_the_merge_class():
    g = _Ctx({"step": (50.0, 25, dict(_COV, steps=2500)), "merge": (34.0, 2500,
                                                                    dict(_COV, steps=2500))})
    kind, ms, n, cov, other = bench.whole_step_class(g, "step")
    assert kind == "step" and ms == 50.0 and n == 25
    m = other["merge_class"]
    assert m["launches"] == 2500 and m["avg_launch_ms"] == pytest.approx(34.0 / 2500)
    assert m["algorithmic_bytes_per_launch"] == pytest.approx(
        bench.algorithmic_bytes("merge", dict(_COV, steps=2500)) / 2500)


def test_traffic_only_for_the_profiled_steps_and_sources(tmp_path, monkeypatch):
    """The committed counter bytes of a kernel class are printed only while the class's own
    sources are the ones profiled and the timed launches cover as many steps each; a change to
    another class's sources leaves them valid."""
    for rel in {r for v in bench.KERNEL_SOURCES.values() for r in v}:
        f = tmp_path / rel
        f.parent.mkdir(parents=True, exist_ok=True)
        f.write_text("source of " + rel)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    summary = tmp_path / "profiles" / "k_persist_ghz20_nm_traffic.md"
    summary.write_text("hbm_bytes_per_launch: 1.5e+09\nsteps_per_launch: 1777\n"
                       f"sources_digest: {bench.sources_digest('fused')}\n")
    assert bench.profiled_traffic("fused", "ghz20_nm", 1777.0) == 1.5e9
    assert bench.profiled_traffic("fused", "ghz20_nm", 20.0) is None
    assert bench.profiled_traffic("fused", "dd12", 1777.0) is None
    (tmp_path / "paper_2502_18929_amd/csrc/qmc_small.hip").write_text("changed")
    assert bench.profiled_traffic("fused", "ghz20_nm", 1777.0) == 1.5e9
    (tmp_path / "paper_2502_18929_amd/csrc/qmc_host.cpp").write_text("changed")
    assert bench.profiled_traffic("fused", "ghz20_nm", 1777.0) is None
