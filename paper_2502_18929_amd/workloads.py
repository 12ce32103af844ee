"""Seeded synthetic workloads shaped like the circuits of Shen & Lidar, arXiv:2502.18929.

This module only *describes problems*: Pauli-monomial models of eq. (1), per-step weights
s_m(t_s) and gamma_k(t_s) at the left end of each step, ideal pulse schedules, initial integer
records N(0) = N^diag rho(0) (eq. (3) paragraph) and observables.  It holds none of the method's
arithmetic, so both the HIP library and the CPU oracle can be fed from it.

Conventions: qubit q of |i> is bit q of i; a monomial (x, z, c) is c * X^x Z^z with
X^x Z^z |i> = (-1)^popcount(z & i) |i ^ x>; the element |i><j| has key (j << n) | i.

Workloads (paper section in brackets):
* ``ghz``: noisy GHZ preparation [Markovian circuit dynamics, Fig. 1(d)]: a Hadamard on qubit 0
  during [0, 1) as (pi/2)(X+Z)/sqrt(2), then CNOT(k-1 -> k) during [k, k+1) as
  (pi/4)(I - Z_c - X_t + Z_c X_t) (identity dropped); dephasing L = Z_q and damping
  L = sigma^-_q = (X_q - X_q Z_q)/2 on every qubit (|0> is the ground state).  Optionally a
  non-Markovian dephasing rate gamma(t) = a cos(w t) that goes negative [Non-Markovian dynamics].
* ``dd``: staggered-XX dynamical decoupling with ZZ crosstalk on a ring [Fig. 1(c)], simulated in
  the Pauli-X basis where |+>^n is the single key 0 [text after Fig. 2]; X pulses are ideal and
  instantaneous (X_q becomes Z_q in that frame), even qubits at tau/2 + k tau, odd at (k+1) tau.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    n: int
    n_replicas: int
    seed: int
    dt: float
    nsteps: int
    walker_target: int
    h: list                     # [(x, z, coeff)], H(t) = sum_m s_m(t) h_m
    lops: list                  # [[(x, z, coeff), ...]] one list per Lindblad operator L_k
    s: np.ndarray               # [nsteps, n_h] weights s_m(t_s)
    gamma: np.ndarray           # [nsteps, n_l] rates gamma_k(t_s)
    init_keys: np.ndarray
    init_re: np.ndarray
    init_im: np.ndarray
    pulses: dict = field(default_factory=dict)   # {step: [(x, z)]} applied before that step
    pauli_obs: list = field(default_factory=list)  # [(label, x, z, phase)]
    psi: list = field(default_factory=list)        # sparse |psi>: [(index, amplitude)]
    frame: str = "Z"
    notes: str = ""
    step_dt: np.ndarray | None = None  # physical time step of every step (None: dt throughout)

    @property
    def n_h(self):
        return len(self.h)

    @property
    def n_l(self):
        return len(self.lops)

    def pulse_steps(self):
        return sorted(self.pulses)

    def segments(self):
        """Split [0, nsteps) into runs of steps between pulses: [(start, stop, pulses_before)]."""
        cuts = sorted(set([0, self.nsteps] + [k for k in self.pulses if 0 < k < self.nsteps]))
        out = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            out.append((a, b, self.pulses.get(a, [])))
        return out

    def truncated(self, nsteps: int, n_replicas: int | None = None, walker_target=None):
        """The same workload cut to its first nsteps (and optionally fewer replicas/walkers)."""
        w = Workload(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        w.nsteps = nsteps
        w.s = self.s[:nsteps].copy()
        w.gamma = self.gamma[:nsteps].copy()
        w.pulses = {k: v for k, v in self.pulses.items() if k <= nsteps}
        if self.step_dt is not None:
            w.step_dt = self.step_dt[:nsteps].copy()
        if n_replicas is not None:
            w.n_replicas = n_replicas
        if walker_target is not None:
            w.walker_target = int(walker_target)
            w.init_re = np.array([int(walker_target)], dtype=np.int32)
        return w


def _bit(q):
    return 1 << q


def _single_key_init(target):
    return (np.array([0], dtype=np.uint64), np.array([int(target)], dtype=np.int32),
            np.array([0], dtype=np.int32))


def ghz(n=4, n_replicas=4, walker_target=10_000, dt=0.01, n_gates=None, seed=1,
        gamma_deph=0.01, gamma_damp=0.005, deph_cos=None, name=None):
    """Noisy GHZ preparation.  n_gates = number of unit-time gate windows (Hadamard + CNOTs);
    by default n (Hadamard plus n-1 CNOTs).  deph_cos = (a, w) makes the dephasing rate
    a*cos(w t) (non-Markovian when negative); otherwise gamma_deph is constant."""
    if n_gates is None:
        n_gates = n
    steps_per_unit = int(round(1.0 / dt))
    assert abs(steps_per_unit * dt - 1.0) < 1e-12, "dt must divide the unit gate time"
    nsteps = n_gates * steps_per_unit
    h, seg = [], []
    a = math.pi / (2.0 * math.sqrt(2.0))
    h += [(_bit(0), 0, a), (0, _bit(0), a)]
    seg += [0, 0]
    for k in range(1, n_gates):
        c, t = k - 1, k
        q = math.pi / 4.0
        h += [(0, _bit(c), -q), (_bit(t), 0, -q), (_bit(t), _bit(c), q)]
        seg += [k, k, k]
    lops = [[(0, _bit(q), 1.0)] for q in range(n)]
    lops += [[(_bit(q), 0, 0.5), (_bit(q), _bit(q), -0.5)] for q in range(n)]
    s = np.zeros((nsteps, len(h)))
    gamma = np.zeros((nsteps, len(lops)))
    for k in range(nsteps):
        unit = k // steps_per_unit
        for m, sg in enumerate(seg):
            if sg == unit:
                s[k, m] = 1.0
        t = k * dt
        gd = gamma_deph if deph_cos is None else deph_cos[0] * math.cos(deph_cos[1] * t)
        gamma[k, :n] = gd
        gamma[k, n:] = gamma_damp
    keys, re, im = _single_key_init(walker_target)
    m = n_gates  # qubits entangled by the end of the circuit
    ghz_hi = (1 << m) - 1
    amp = 1.0 / math.sqrt(2.0)
    pauli_obs = [(f"Z{q}", 0, _bit(q), 1.0) for q in range(n)]
    return Workload(name=name or f"ghz_n{n}", n=n, n_replicas=n_replicas, seed=seed, dt=dt,
                    nsteps=nsteps, walker_target=walker_target, h=h, lops=lops, s=s,
                    gamma=gamma, init_keys=keys, init_re=re, init_im=im, pauli_obs=pauli_obs,
                    psi=[(0, amp), (ghz_hi, amp)], frame="Z",
                    notes=f"GHZ on the first {m} qubits at the end")


def _to_x_frame(mono):
    """Hadamard conjugation of c X^x Z^z: H^n X^x Z^z H^n = Z^x X^z = (-1)^popc(x&z) X^z Z^x."""
    x, z, c = mono
    sign = -1.0 if bin(x & z).count("1") & 1 else 1.0
    return (z, x, sign * c)


def dd(n=12, n_replicas=16, walker_target=1_000_000, dt=0.005, nsteps=4000, seed=2,
       j_scale=0.02, gamma_deph=0.005, gamma_damp=0.002, tau=1.0, disorder_seed=2,
       pulse_width=None, substeps=10, name=None):
    """Staggered-XX dynamical decoupling of |+>^n on a ring with ZZ crosstalk, in the X frame.
    J_q = j_scale * U[0.5, 1.5] from numpy PCG64.  The X pulses on the even qubits at tau/2 + k tau
    and on the odd ones at (k + 1) tau are ideal and instantaneous, or, with pulse_width w, square
    pulses a X_q with a = pi / (2 w) (a pi rotation) over [t_p - w/2, t_p + w/2), integrated with
    `substeps` steps of dt / substeps inside the windows (nsteps counts steps of dt before the
    pulses are sub-stepped; a pulse at the end of the run is completed past it).  A step of
    dt / m is a step of dt with every weight and rate divided by m (L is linear in them), so the
    context keeps one dt; step_dt holds each step's physical time step."""
    rng = np.random.Generator(np.random.PCG64(disorder_seed))
    J = j_scale * rng.uniform(0.5, 1.5, size=n)
    h_z = []
    for q in range(n):
        q2 = (q + 1) % n
        if q2 == q:
            continue
        h_z.append((0, _bit(q) | _bit(q2), float(J[q])))
    lops_z = [[(0, _bit(q), 1.0)] for q in range(n)]
    lops_z += [[(_bit(q), 0, 0.5), (_bit(q), _bit(q), -0.5)] for q in range(n)]
    h = [_to_x_frame(m) for m in h_z]
    lops = [[_to_x_frame(m) for m in op] for op in lops_z]
    s = np.ones((nsteps, len(h)))
    gamma = np.zeros((nsteps, len(lops)))
    gamma[:, :n] = gamma_deph
    gamma[:, n:] = gamma_damp
    per_tau = int(round(tau / dt))
    assert per_tau % 2 == 0 and abs(per_tau * dt - tau) < 1e-12
    even = sum(_bit(q) for q in range(0, n, 2))
    odd = sum(_bit(q) for q in range(1, n, 2))
    pulses = {}
    # Physical X_q is Z_q in the X frame.
    for k in range(per_tau // 2, nsteps + 1, per_tau):
        pulses.setdefault(k, []).append((0, even))
    for k in range(per_tau, nsteps + 1, per_tau):
        pulses.setdefault(k, []).append((0, odd))
    # merge pulses at the same step into one Pauli (they commute)
    pulses = {k: [(0, sum(z for _, z in v))] for k, v in pulses.items()}
    step_dt = None
    notes = "X frame, ideal pulses"
    if pulse_width is not None:
        hw = int(round(pulse_width / (2.0 * dt)))
        assert hw >= 1 and abs(2 * hw * dt - pulse_width) < 1e-12, \
            "the pulse width must be an even number of steps"
        assert 2 * hw <= per_tau // 2, "pulse windows must not overlap"
        assert substeps >= 1
        amp = math.pi / (2.0 * pulse_width)
        n_j = len(h)
        h = h + [_to_x_frame((_bit(q), 0, 1.0)) for q in range(n)]  # physical X_q
        # physical qubits pulsed during step k; a pulse centred on the last instant (the ideal
        # pulse after the final step) is completed, so the run ends half a window later
        active = np.zeros(nsteps + hw, dtype=np.int64)
        for k, v in pulses.items():
            for _, z in v:  # the X-frame Z mask of an ideal pulse is its physical X mask
                active[max(0, k - hw):k + hw] |= z
        rows_s, rows_g, sdt = [], [], []
        for k in range(nsteps + hw):
            if k >= nsteps and active[k] == 0:
                break
            kk = min(k, nsteps - 1)
            srow = np.zeros(n_j + n)
            srow[:n_j] = s[kk]
            if active[k] == 0:
                rows_s.append(srow)
                rows_g.append(gamma[kk])
                sdt.append(dt)
                continue
            for q in range(n):
                if (int(active[k]) >> q) & 1:
                    srow[n_j + q] = amp
            for _ in range(substeps):
                rows_s.append(srow / substeps)
                rows_g.append(gamma[kk] / substeps)
                sdt.append(dt / substeps)
        s = np.array(rows_s)
        gamma = np.array(rows_g)
        step_dt = np.array(sdt)
        nsteps = len(sdt)
        pulses = {}
        notes = (f"X frame, square pulses of width {pulse_width} (amplitude {amp:.4g}), "
                 f"steps of dt/{substeps} inside them")
    keys, re, im = _single_key_init(walker_target)
    # <Z_q> in the physical frame is <X_q> in the X frame.
    pauli_obs = [(f"Z{q}", _bit(q), 0, 1.0) for q in range(n)]
    return Workload(name=name or f"dd_n{n}", n=n, n_replicas=n_replicas, seed=seed, dt=dt, nsteps=nsteps,
                    walker_target=walker_target, h=h, lops=lops, s=s, gamma=gamma,
                    init_keys=keys, init_re=re, init_im=im, pulses=pulses, pauli_obs=pauli_obs,
                    psi=[(0, 1.0)], frame="X", notes=notes, step_dt=step_dt)


# ---- the three single-GPU configurations ----------------------------------------------------

def config_ghz4():
    """n=4 noisy GHZ preparation, dt=0.01, 400 steps, 4 replicas x 1e4, Philox seed 1."""
    return ghz(n=4, n_replicas=4, walker_target=10_000, dt=0.01, seed=1, name="ghz4")


def config_dd12(pulse_width=None, substeps=10):
    """n=12 staggered-XX DD with ZZ crosstalk, dt=0.005, 4000 steps, 16 replicas x 1e6; ideal
    pulses, or square pulses of that width with steps of dt / substeps inside them."""
    return dd(n=12, n_replicas=16, walker_target=1_000_000, dt=0.005, nsteps=4000, seed=2,
              pulse_width=pulse_width, substeps=substeps,
              name="dd12" if pulse_width is None else "dd12_finite")


def config_ghz20_nm():
    """n=20 GHZ preparation with non-Markovian dephasing 0.02 cos(0.5 t) and damping 0.002,
    dt=0.005, 3000 steps (15 unit gate windows: Hadamard then CNOTs up to 13->14),
    8 replicas x 1e7 walkers."""
    return ghz(n=20, n_replicas=8, walker_target=10_000_000, dt=0.005, n_gates=15, seed=3,
               gamma_damp=0.002, deph_cos=(0.02, 0.5), name="ghz20_nm")


@dataclass
class BatchWorkload:
    """Many circuits advanced together (one context, one step launch).  Every circuit is a
    Workload on its own n_c <= n qubits; in the batch it lives on n qubits with the extra ones
    idle (its masks and keys only touch its own qubits).  Replica r of circuit c is segment
    c * n_replicas + r."""
    name: str
    n: int
    n_replicas: int
    seed: int
    dt: float
    nsteps: int
    circuits: list

    def weights(self, a, b):
        """Weights of steps [a, b) of all circuits side by side (circuit order)."""
        s = np.concatenate([w.s[a:b] for w in self.circuits], axis=1)
        g = np.concatenate([w.gamma[a:b] for w in self.circuits], axis=1)
        return s, g

    def segments(self):
        """[(start, stop, masks)]: runs of steps between pulse steps of any circuit; masks is
        None or (xs, zs), the Pauli of every circuit before the run (0, 0 = none)."""
        steps = set()
        for w in self.circuits:
            steps |= {k for k in w.pulses if 0 < k < self.nsteps}
        cuts = sorted(steps | {0, self.nsteps})
        out = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            xs = np.zeros(len(self.circuits), dtype=np.uint64)
            zs = np.zeros(len(self.circuits), dtype=np.uint64)
            any_p = False
            for c, w in enumerate(self.circuits):
                for (px, pz) in w.pulses.get(a, []):
                    xs[c] ^= np.uint64(px)
                    zs[c] ^= np.uint64(pz)
                    any_p = True
            out.append((a, b, (xs, zs) if any_p else None))
        return out


def batch(n_circuits=64, n_lo=6, n_hi=16, n_replicas=4, nsteps=1000, dt=0.005, seed=5,
          w_lo=1e4, w_hi=1e6, rate_lo=0.001, rate_hi=0.02, name=None):
    """Batched circuits of uneven size: n_c ~ U{n_lo..n_hi}, each a DD-crosstalk or a GHZ
    circuit (as dd / ghz above) with rates ~ U[rate_lo, rate_hi] and a walker target
    log-uniform in [w_lo, w_hi], drawn from numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    circuits = []
    units = int(math.ceil(nsteps * dt - 1e-9))
    for c in range(n_circuits):
        nc = int(rng.integers(n_lo, n_hi + 1))
        kind = "dd" if rng.random() < 0.5 else "ghz"
        g1, g2 = (float(x) for x in rng.uniform(rate_lo, rate_hi, size=2))
        wt = int(round(math.exp(rng.uniform(math.log(w_lo), math.log(w_hi)))))
        if kind == "dd":
            w = dd(n=nc, n_replicas=n_replicas, walker_target=wt, dt=dt, nsteps=nsteps,
                   seed=seed, gamma_deph=g1, gamma_damp=g2, disorder_seed=seed * 1000 + c)
        else:
            w = ghz(n=nc, n_replicas=n_replicas, walker_target=wt, dt=dt,
                    n_gates=max(1, min(nc, units)), seed=seed, gamma_deph=g1, gamma_damp=g2)
            w = w.truncated(nsteps) if w.nsteps > nsteps else w
            if w.nsteps < nsteps:  # idle after the last gate, the noise going on
                extra = nsteps - w.nsteps
                w.s = np.concatenate([w.s, np.zeros((extra, w.n_h))])
                w.gamma = np.concatenate([w.gamma, np.repeat(w.gamma[-1:], extra, axis=0)])
                w.nsteps = nsteps
        w.name = f"{kind}_n{nc}_c{c}"
        circuits.append(w)
    n = max(w.n for w in circuits)
    return BatchWorkload(name=name or f"batch{n_circuits}", n=n, n_replicas=n_replicas,
                         seed=seed, dt=dt, nsteps=nsteps, circuits=circuits)


def config_batch64():
    """64 circuits, n ~ U{6..16}, DD or GHZ, rates U[0.001, 0.02], walker targets log-uniform
    in 1e4..1e6, 4 replicas each, dt = 0.005, 1000 steps (the batched configuration)."""
    return batch(name="batch64")


CONFIGS = {"ghz4": config_ghz4, "dd12": config_dd12, "ghz20_nm": config_ghz20_nm}


# ---- random models for unit tests -------------------------------------------------------------

def random_model(n, rng, n_h=4, n_l=2, max_l_terms=2):
    """Random Hermitian-coefficient H monomials and random Lindblad operators."""
    D = 1 << n
    h = []
    for _ in range(n_h):
        x, z = int(rng.integers(D)), int(rng.integers(D))
        c = rng.normal()
        if bin(x & z).count("1") & 1:   # X^x Z^z is anti-Hermitian: Hermitian needs i*c
            c = 1j * c
        h.append((x, z, c))
    lops = []
    for _ in range(n_l):
        k = int(rng.integers(1, max_l_terms + 1))
        lops.append([(int(rng.integers(D)), int(rng.integers(D)),
                      complex(rng.normal(), rng.normal())) for _ in range(k)])
    return h, lops


def random_mlp(rng, hidden_shift=5, scale=40):
    """Seeded weights of the spawn-proposal MLP (shapes of the C ABI: w1 int8 [32, 64], b1 int32
    [32], w2 int8 [64, 32], b2 int32 [64], hidden shift): random inputs, not trained ones."""
    w1 = rng.integers(-scale, scale + 1, size=(32, 64)).astype(np.int8)
    b1 = rng.integers(-200, 800, size=32).astype(np.int32)
    w2 = rng.integers(-scale, scale + 1, size=(64, 32)).astype(np.int8)
    b2 = rng.integers(-2000, 4000, size=64).astype(np.int32)
    return w1, b1, w2, b2, int(hidden_shift)


def random_deep_mlp(rng, s1=6, s2=9, scale=40):
    """Seeded weights of the deeper spawn-proposal network (shapes of the C ABI: w1 int8 [128, 128],
    b1 int32 [128], w2 int8 [128, 128], b2 int32 [128], w3 int8 [64, 128], b3 int32 [64], hidden
    shifts s1, s2): random inputs, not trained ones."""
    w1 = rng.integers(-scale, scale + 1, size=(128, 128)).astype(np.int8)
    b1 = rng.integers(-200, 800, size=128).astype(np.int32)
    w2 = rng.integers(-scale, scale + 1, size=(128, 128)).astype(np.int8)
    b2 = rng.integers(-500, 3000, size=128).astype(np.int32)
    w3 = rng.integers(-scale, scale + 1, size=(64, 128)).astype(np.int8)
    b3 = rng.integers(-2000, 6000, size=64).astype(np.int32)
    return w1, b1, w2, b2, w3, b3, int(s1), int(s2)


def random_records(n, rng, count, scale=50):
    """Sorted unique keys over 2n bits with nonzero Gaussian-integer populations."""
    K = 1 << (2 * n)
    count = min(count, K)
    keys = np.sort(rng.choice(K, size=count, replace=False)).astype(np.uint64)
    re = rng.integers(-scale, scale + 1, size=count).astype(np.int32)
    im = rng.integers(-scale, scale + 1, size=count).astype(np.int32)
    zero = (re == 0) & (im == 0)
    re[zero] = 1
    return keys, re, im
