"""Writes ghz4_exact.json: the dense solutions of the ghz4 workload (n = 4 noisy GHZ preparation,
dt = 0.01, 400 steps) at the end of the circuit, from oracle/dense.py only.

For each of three dense propagations of the column-stacked master equation (eqs. (1)-(2)) -- the
Euler map and the AB2 map of the End Matter on simulation methodology (the exact expectations of
the stochastic Euler and AB2 steps, by linearity) and the exact piecewise exponential (the
physical solution the paper's Fig. 2(a) compares with) -- it stores <Z_q>, the GHZ fidelity and the
trace of rho(t_f).  bench.py reads the file to state how far the GPU replica means lie from each.

Run: python tests/golden/make_exact.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def observables(v, w):
    from oracle import dense as D
    rho = D.unvec(v, w.n)
    out = {"trace": float(np.trace(rho).real)}
    for label, x, z, ph in w.pauli_obs:
        out[label] = float((complex(ph) * np.trace(D.pauli(w.n, x, z) @ rho)).real)
    psi = np.zeros(1 << w.n, dtype=complex)
    for idx, amp in w.psi:
        psi[idx] = amp
    out["fidelity"] = float((psi.conj() @ rho @ psi).real)
    return out


def exact_values():
    from oracle import dense as D
    from paper_2502_18929_amd import workloads as W
    w = W.config_ghz4()
    assert not w.pulses
    m = D.DenseModel(w.n, w.h, w.lops)
    v0 = np.zeros(1 << (2 * w.n), dtype=complex)
    for k, a, b in zip(w.init_keys, w.init_re, w.init_im):
        v0[int(k)] = complex(int(a), int(b)) / float(w.walker_target)
    return {
        "workload": w.name, "nsteps": int(w.nsteps), "dt": w.dt,
        "euler_map": observables(D.euler_map(m, w.s, w.gamma, w.dt, v0), w),
        "ab2_map": observables(D.ab2_map(m, w.s, w.gamma, w.dt, v0), w),
        "expm": observables(D.expm_piecewise(m, w.s, w.gamma, w.dt, v0), w),
    }


if __name__ == "__main__":
    vals = exact_values()
    with open(os.path.join(HERE, "ghz4_exact.json"), "w") as f:
        json.dump(vals, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(vals, indent=1))
