"""Dense reference for the master equation of Shen & Lidar, arXiv:2502.18929, eqs. (1)-(2).

TEST INFRASTRUCTURE ONLY (see the package docstring).  For n <= 5 qubits this builds the full
D^2 x D^2 Liouvillian with Kronecker products and integrates it:

* ``liouvillian``: eq. (2) in the standard (conjugated) form, for column-stacked vec(rho), so that
  the element |i><j| sits at index j*D + i (the same layout as the walker keys);
* ``euler_map``: the dense first-order Euler map of the End Matter on simulation methodology --
  the exact expectation of the stochastic Euler step, by linearity;
* ``ab2_map``: the second-order Adams-Bashforth map of the same paragraph;
* ``rk4`` and ``expm_piecewise``: accurate integrators for the physical solution.

Qubit q of basis state |i> is bit q of i.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pauli(n: int, x: int, z: int) -> np.ndarray:
    """Dense X^x Z^z: |i> -> (-1)^popcount(z & i) |i ^ x>."""
    D = 1 << n
    M = np.zeros((D, D), dtype=complex)
    for i in range(D):
        M[i ^ x, i] = -1.0 if bin(z & i).count("1") & 1 else 1.0
    return M


def operator(n: int, monos) -> np.ndarray:
    """Sum of c * X^x Z^z over the (x, z, c) monomials."""
    D = 1 << n
    M = np.zeros((D, D), dtype=complex)
    for x, z, c in monos:
        M += complex(c) * pauli(n, int(x), int(z))
    return M


def liouvillian(n: int, H: np.ndarray, lops) -> np.ndarray:
    """Column-stacked Liouvillian of eq. (1): lops is a list of (gamma_k, L_k dense).

    vec(A rho B) = (B^T kron A) vec(rho) for column stacking, so
    -i H rho -> -i (I kron H),  +i rho H -> +i (H^T kron I),
    gamma L rho L^dag -> gamma (conj(L) kron L),
    -(gamma/2){L^dag L, rho} -> -(gamma/2) (I kron L^dag L + (L^dag L)^T kron I).
    """
    D = 1 << n
    Id = np.eye(D)
    Lv = -1j * np.kron(Id, H) + 1j * np.kron(H.T, Id)
    for g, L in lops:
        LdL = L.conj().T @ L
        Lv = Lv + g * (np.kron(L.conj(), L) - 0.5 * np.kron(Id, LdL) - 0.5 * np.kron(LdL.T, Id))
    return Lv


class DenseModel:
    """Dense operators of a model given as H monomials and Lindblad monomial lists."""

    def __init__(self, n, h, lops):
        self.n = n
        self.Hm = [operator(n, [m]) for m in h]
        self.Lk = [operator(n, op) for op in lops]

    def L(self, s, gamma):
        D = 1 << self.n
        H = np.zeros((D, D), dtype=complex)
        for w, Hm in zip(s, self.Hm):
            if w != 0.0:
                H = H + w * Hm
        return liouvillian(self.n, H, [(g, L) for g, L in zip(gamma, self.Lk)])


def vec(rho: np.ndarray) -> np.ndarray:
    return rho.reshape(-1, order="F")


def unvec(v: np.ndarray, n: int) -> np.ndarray:
    D = 1 << n
    return v.reshape(D, D, order="F")


def euler_map(model: DenseModel, s_seq, g_seq, dt, v0, pulses=None, record=None):
    """v_{k+1} = v_k + dt L(t_k) v_k for every step k (End Matter, Euler solver).

    pulses: optional {step: [dense superoperator]} applied before that step (a step equal to
    the number of steps means after the last one).  record(k, v) is called after each step."""
    v = np.array(v0, dtype=complex)
    cache = {}
    nsteps = len(s_seq) if len(s_seq) else len(g_seq)
    for k in range(nsteps):
        if pulses and k in pulses:
            for P in pulses[k]:
                v = P @ v
        key = (tuple(s_seq[k]) if len(s_seq) else (), tuple(g_seq[k]) if len(g_seq) else ())
        if key not in cache:
            cache[key] = model.L(s_seq[k] if len(s_seq) else [], g_seq[k] if len(g_seq) else [])
        v = v + dt * (cache[key] @ v)
        if record is not None:
            record(k, v)
    if pulses and nsteps in pulses:
        for P in pulses[nsteps]:
            v = P @ v
    return v


def ab2_map(model: DenseModel, s_seq, g_seq, dt, v0):
    """AB2 (End Matter): v_{k+2} = v_{k+1} + dt [3/2 L_{k+1} v_{k+1} - 1/2 L_k v_k], first step Euler."""
    v = np.array(v0, dtype=complex)
    prev = None
    for k in range(len(s_seq)):
        f = model.L(s_seq[k], g_seq[k]) @ v
        v = v + dt * f if prev is None else v + dt * (1.5 * f - 0.5 * prev)
        prev = f
    return v


def rk4(model: DenseModel, s_fn, g_fn, dt, nsteps, v0, record=None):
    """Classical RK4 with H(t), gamma(t) evaluated at the stage times."""
    v = np.array(v0, dtype=complex)
    for k in range(nsteps):
        t = k * dt
        L0 = model.L(s_fn(t), g_fn(t))
        Lh = model.L(s_fn(t + dt / 2), g_fn(t + dt / 2))
        L1 = model.L(s_fn(t + dt), g_fn(t + dt))
        k1 = L0 @ v
        k2 = Lh @ (v + dt / 2 * k1)
        k3 = Lh @ (v + dt / 2 * k2)
        k4 = L1 @ (v + dt * k3)
        v = v + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if record is not None:
            record(k, v)
    return v


def expm_piecewise(model: DenseModel, s_seq, g_seq, dt, v0):
    """Exact propagation when H and gamma are constant over each step (left-endpoint values)."""
    v = np.array(v0, dtype=complex)
    cache = {}
    for k in range(len(s_seq)):
        key = (tuple(s_seq[k]), tuple(g_seq[k]))
        if key not in cache:
            cache[key] = sla.expm(dt * model.L(s_seq[k], g_seq[k]))
        v = cache[key] @ v
    return v


def pulse_superop(n: int, x: int, z: int) -> np.ndarray:
    """rho -> P rho P^dagger for P = X^x Z^z, as a dense superoperator on vec(rho)."""
    P = pauli(n, x, z)
    return np.kron(P.conj(), P)
