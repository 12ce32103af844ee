"""The stored dense solutions of ghz4 (tests/golden/ghz4_exact.json, read by bench.py to state the
GPU replica means against the exact result) are what their committed script computes from the
dense reference, and they carry the integrators' known time-step biases (End Matter on
simulation methodology: Euler first order, AB2 second order)."""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def test_stored_exact_values_are_current():
    import make_exact
    stored = json.load(open(os.path.join(HERE, "golden", "ghz4_exact.json")))
    fresh = make_exact.exact_values()
    assert stored["workload"] == fresh["workload"] and stored["nsteps"] == fresh["nsteps"]
    for m in ("euler_map", "ab2_map", "expm"):
        for k, v in fresh[m].items():
            assert stored[m][k] == pytest.approx(v, abs=1e-12), (m, k)


def test_stored_exact_values_show_the_integrator_biases():
    v = json.load(open(os.path.join(HERE, "golden", "ghz4_exact.json")))
    e = max(abs(v["euler_map"][k] - v["expm"][k]) for k in v["expm"])
    a = max(abs(v["ab2_map"][k] - v["expm"][k]) for k in v["expm"])
    assert 0.05 < e < 0.2          # Euler at dt = 0.01: about 0.10 in <Z_3>
    assert a < 0.01 and a < e / 10  # AB2: about 8e-4
    for m in ("euler_map", "ab2_map", "expm"):
        assert v[m]["trace"] == pytest.approx(1.0, abs=1e-12)   # trace preserving
    assert v["expm"]["fidelity"] == pytest.approx(0.9051, abs=1e-4)
