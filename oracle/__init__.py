"""CPU oracle for the real-time QMC step of Shen & Lidar, arXiv:2502.18929.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check and by the
CPU-baseline leg of ``bench.py``; never by the product path.  It shares no code with the HIP
library: ``qmc_oracle.c`` is its own Philox, Liouvillian term compiler, quantizer, step and
estimators, and ``dense.py`` holds dense reference integrators.  This module only marshals
arguments into the C oracle with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

ORC_OK = 0
ORC_ERR_ARG = -1
ORC_ERR_DT = -2
ORC_ERR_COUNT_OVERFLOW = -5


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (fixed FP64 operation order: no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
               "-ffp-contract=off", "-fopenmp", os.path.join(_HERE, "qmc_oracle.c"),
               "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Mono(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint64), ("z", ctypes.c_uint64),
                ("re", ctypes.c_double), ("im", ctypes.c_double)]


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u32, u64, i32, i64, dbl = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                                   ctypes.c_int64, ctypes.c_double)
        P = ctypes.POINTER
        L.orc_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.orc_philox4x32_10.restype = None
        L.orc_comb.argtypes = [u32, P(i64), u32, P(i64)]
        L.orc_comb.restype = None
        L.orc_create.argtypes = [u32, u32, u64, dbl, u32, P(_Mono), u32, P(u32), P(_Mono),
                                 P(u64), P(i32), P(i32), u64, P(ctypes.c_void_p)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_destroy.restype = None
        L.orc_n_terms.argtypes = [ctypes.c_void_p]
        L.orc_n_terms.restype = u32
        L.orc_get_terms.argtypes = [ctypes.c_void_p, P(u64), P(u64), P(dbl), P(dbl), P(u32),
                                    P(u32)]
        L.orc_table.argtypes = [ctypes.c_void_p, P(dbl), P(dbl), dbl, u32, u32, P(u32), P(u64),
                                P(u32), P(u32), P(u64), P(i64)]
        L.orc_column_fp.argtypes = [ctypes.c_void_p, P(dbl), P(dbl), u64, u32, P(u32), P(u64),
                                    P(dbl)]
        L.orc_column_q.argtypes = [ctypes.c_void_p, P(dbl), P(dbl), dbl, u64, u32, P(u32), P(u64),
                                   P(i64)]
        L.orc_step.argtypes = [ctypes.c_void_p, u32, P(dbl), P(dbl)]
        L.orc_step_threads.argtypes = [ctypes.c_void_p, u32, P(dbl), P(dbl), ctypes.c_int,
                                       P(ctypes.c_int)]
        L.orc_pulse.argtypes = [ctypes.c_void_p, u64, u64]
        L.orc_set_shift.argtypes = [ctypes.c_void_p, u32, dbl]
        L.orc_get_shift.argtypes = [ctypes.c_void_p, u32]
        L.orc_get_shift.restype = dbl
        L.orc_set_shift_control.argtypes = [ctypes.c_void_p, ctypes.c_int, dbl, u32, u64]
        L.orc_set_initiator.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.orc_set_replica_base.argtypes = [ctypes.c_void_p, u32]
        i8p = P(ctypes.c_int8)
        L.orc_set_proposal.argtypes = [ctypes.c_void_p, u32, u32, i8p, P(ctypes.c_int32), i8p,
                                       P(ctypes.c_int32), u32]
        L.orc_mlp_scores.argtypes = [ctypes.c_void_p, u64, P(ctypes.c_int32)]
        L.orc_set_proposal_deep.argtypes = [ctypes.c_void_p, u32, i8p, P(ctypes.c_int32), i8p,
                                            P(ctypes.c_int32), i8p, P(ctypes.c_int32), u32, u32]
        L.orc_deep_scores.argtypes = [ctypes.c_void_p, u64, P(u64), P(ctypes.c_int32)]
        L.orc_step_active.argtypes = [ctypes.c_void_p, P(dbl), P(dbl), P(u64)]
        L.orc_proposal_thresholds.argtypes = [u32, P(u64), P(u64)]
        L.orc_proposal_draw.argtypes = [u32, P(i64), P(u64), u32, u32, u32, P(u32), P(i64)]
        L.orc_counters.argtypes = [ctypes.c_void_p, P(u64), P(u64), P(u64), P(u64)]
        L.orc_counters.restype = None
        L.orc_get_step.argtypes = [ctypes.c_void_p]
        L.orc_get_step.restype = u32
        L.orc_size.argtypes = [ctypes.c_void_p, u32]
        L.orc_size.restype = u64
        L.orc_export.argtypes = [ctypes.c_void_p, u32, P(u64), P(i32), P(i32), u64, P(u64)]
        L.orc_import.argtypes = [ctypes.c_void_p, u32, P(u64), P(i32), P(i32), u64, u32]
        L.orc_set_integrator.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_prev.argtypes = [ctypes.c_void_p, u32, P(u64), P(i32), P(i32), u64, P(dbl),
                                   P(dbl)]
        L.orc_export_prev.argtypes = [ctypes.c_void_p, u32, P(u64), P(i32), P(i32), u64,
                                      P(u64)]
        L.orc_observe.argtypes = [ctypes.c_void_p, u32, u32, P(u64), P(u64), u32, P(u64),
                                  P(u64), P(u64), P(i64), P(i64), P(i64), P(u64)]
        _lib = L
    return _lib


MLP_IN, MLP_HIDDEN, MLP_OUT = 64, 32, 64
DEEP_IN, DEEP_HIDDEN, DEEP_OUT = 128, 128, 64


def proposal_thresholds(W):
    """Thresholds P (sum 2^32, each >= 1) from the nonnegative integer weights W (reading R18)."""
    W = np.ascontiguousarray(W, dtype=np.uint64)
    P = np.zeros(len(W), dtype=np.uint64)
    _check(lib().orc_proposal_thresholds(len(W), _p(W, ctypes.c_uint64), _p(P, ctypes.c_uint64)),
           "proposal_thresholds")
    return P


def proposal_draw(x, P, K, u, j):
    """One proposal draw (reading R18): (channel, signed walkers) for uniforms u (32 bits) and
    j < K."""
    x = np.ascontiguousarray(x, dtype=np.int64)
    P = np.ascontiguousarray(P, dtype=np.uint64)
    ch, n = ctypes.c_uint32(), ctypes.c_int64()
    _check(lib().orc_proposal_draw(len(x), _p(x, ctypes.c_int64), _p(P, ctypes.c_uint64), int(K),
                                   int(u), int(j), ctypes.byref(ch), ctypes.byref(n)),
           "proposal_draw")
    return int(ch.value), int(n.value)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32),
                            _p(o, ctypes.c_uint32))
    return o


def comb(x, U):
    x = np.ascontiguousarray(x, dtype=np.int64)
    o = np.zeros_like(x)
    lib().orc_comb(len(x), _p(x, ctypes.c_int64), int(U) & 0xFFFFFFFF, _p(o, ctypes.c_int64))
    return o


def _monos(lst):
    arr = (_Mono * max(1, len(lst)))()
    for i, (x, z, c) in enumerate(lst):
        c = complex(c)
        arr[i] = _Mono(int(x), int(z), c.real, c.imag)
    return arr


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def _check(rc, what):
    if rc != ORC_OK:
        raise OracleError(rc, what)


class Oracle:
    """One oracle context: n qubits, R replicas, the model, and the initial records."""

    def __init__(self, n, n_replicas, seed, dt, h, lops, keys, re, im, integrator="euler"):
        """h: list of (x, z, coeff); lops: list of lists of (x, z, coeff) (one list per L_k);
        integrator: "euler" or "ab2" (End Matter on simulation methodology)."""
        self.n, self.R, self.n_h, self.n_l = int(n), int(n_replicas), len(h), len(lops)
        hm = _monos(h)
        flat = [m for op in lops for m in op]
        lm = _monos(flat)
        off = np.zeros(len(lops) + 1, dtype=np.uint32)
        for k, op in enumerate(lops):
            off[k + 1] = off[k] + len(op)
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        re = np.ascontiguousarray(re, dtype=np.int32)
        im = np.ascontiguousarray(im, dtype=np.int32)
        self._ctx = ctypes.c_void_p()
        _check(lib().orc_create(self.n, self.R, int(seed), float(dt), len(h), hm, len(lops),
                                _p(off, ctypes.c_uint32), lm, _p(keys, ctypes.c_uint64),
                                _p(re, ctypes.c_int32), _p(im, ctypes.c_int32), len(keys),
                                ctypes.byref(self._ctx)), "create")
        if integrator != "euler":
            _check(lib().orc_set_integrator(self._ctx, {"ab2": 1}[integrator]), "integrator")

    def close(self):
        if self._ctx:
            lib().orc_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- model -------------------------------------------------------------------------------
    def terms(self):
        n = lib().orc_n_terms(self._ctx)
        xm = np.zeros(n, np.uint64); zm = np.zeros(n, np.uint64)
        kr = np.zeros(n); ki = np.zeros(n)
        kind = np.zeros(n, np.uint32); idx = np.zeros(n, np.uint32)
        lib().orc_get_terms(self._ctx, _p(xm, ctypes.c_uint64), _p(zm, ctypes.c_uint64),
                            _p(kr, ctypes.c_double), _p(ki, ctypes.c_double),
                            _p(kind, ctypes.c_uint32), _p(idx, ctypes.c_uint32))
        return dict(xmask=xm, zmask=zm, kappa=kr + 1j * ki, kind=kind, index=idx)

    def _w(self, s, gamma):
        s = np.ascontiguousarray(s if self.n_h else np.zeros(1), dtype=np.float64)
        g = np.ascontiguousarray(gamma if self.n_l else np.zeros(1), dtype=np.float64)
        return s, g

    def table(self, s, gamma, scale=1.0):
        s, g = self._w(s, gamma)
        cap_t = lib().orc_n_terms(self._ctx) + 1
        ng = ctypes.c_uint32(); nt = ctypes.c_uint32()
        gx = np.zeros(cap_t + 1, np.uint64); gs = np.zeros(cap_t + 2, np.uint32)
        tz = np.zeros(cap_t, np.uint64); tq = np.zeros((cap_t, 2), np.int64)
        _check(lib().orc_table(self._ctx, _p(s, ctypes.c_double), _p(g, ctypes.c_double),
                               float(scale), cap_t + 1, cap_t, ctypes.byref(ng), _p(gx, ctypes.c_uint64),
                               _p(gs, ctypes.c_uint32), ctypes.byref(nt),
                               _p(tz, ctypes.c_uint64), _p(tq, ctypes.c_int64)), "table")
        G, T = ng.value, nt.value
        return dict(gxmask=gx[:G].copy(), gstart=gs[:G + 1].copy(), zmask=tz[:T].copy(),
                    q=tq[:T].copy())

    def column_fp(self, s, gamma, key):
        s, g = self._w(s, gamma)
        cap = lib().orc_n_terms(self._ctx) + 1
        n = ctypes.c_uint32(); tk = np.zeros(cap, np.uint64); v = np.zeros((cap, 2))
        _check(lib().orc_column_fp(self._ctx, _p(s, ctypes.c_double), _p(g, ctypes.c_double),
                                   int(key), cap, ctypes.byref(n), _p(tk, ctypes.c_uint64),
                                   _p(v, ctypes.c_double)), "column_fp")
        m = n.value
        return tk[:m].copy(), v[:m, 0] + 1j * v[:m, 1]

    def column_q(self, s, gamma, key, scale=1.0):
        s, g = self._w(s, gamma)
        cap = lib().orc_n_terms(self._ctx) + 1
        n = ctypes.c_uint32(); tk = np.zeros(cap, np.uint64); v = np.zeros((cap, 2), np.int64)
        _check(lib().orc_column_q(self._ctx, _p(s, ctypes.c_double), _p(g, ctypes.c_double),
                                  float(scale), int(key), cap, ctypes.byref(n), _p(tk, ctypes.c_uint64),
                                  _p(v, ctypes.c_int64)), "column_q")
        m = n.value
        return tk[:m].copy(), v[:m].copy()

    # -- dynamics ----------------------------------------------------------------------------
    def step(self, s, gamma, threads=1):
        """s: [nsteps, n_h], gamma: [nsteps, n_l]."""
        s = np.asarray(s, dtype=np.float64)
        g = np.asarray(gamma, dtype=np.float64)
        if s.ndim == 2:
            nsteps = s.shape[0]
        elif g.ndim == 2:
            nsteps = g.shape[0]
        else:
            nsteps = s.size // self.n_h if self.n_h else g.size // max(self.n_l, 1)
        s = np.ascontiguousarray(s.reshape(nsteps, self.n_h) if self.n_h
                                 else np.zeros((nsteps, 1)))
        g = np.ascontiguousarray(g.reshape(nsteps, self.n_l) if self.n_l
                                 else np.zeros((nsteps, 1)))
        used = ctypes.c_int(1)
        if threads == 1:
            rc = lib().orc_step(self._ctx, nsteps, _p(s, ctypes.c_double),
                                _p(g, ctypes.c_double))
        else:
            rc = lib().orc_step_threads(self._ctx, nsteps, _p(s, ctypes.c_double),
                                        _p(g, ctypes.c_double), int(threads), ctypes.byref(used))
        _check(rc, "step")
        return used.value

    def pulse(self, x, z):
        _check(lib().orc_pulse(self._ctx, int(x), int(z)), "pulse")

    def set_shift(self, replica, shift):
        _check(lib().orc_set_shift(self._ctx, int(replica), float(shift)), "set_shift")

    def shift(self, replica):
        return lib().orc_get_shift(self._ctx, int(replica))

    def set_shift_control(self, mode, zeta=0.0, period=1, target=0):
        """Variable shift (FCIQMC background paragraph; Booth et al. 2009): mode 1 = on."""
        _check(lib().orc_set_shift_control(self._ctx, int(mode), float(zeta), int(period),
                                           int(target)), "set_shift_control")

    def set_replica_base(self, base):
        """Philox stream ids base .. base + R - 1 for this context's replicas (one circuit of a
        batch of circuits)."""
        _check(lib().orc_set_replica_base(self._ctx, int(base)), "set_replica_base")

    def set_initiator(self, min_walkers):
        """Initiator approximation (End Matter on simulation methodology, reading R17): parents
        with |re| + |im| < min_walkers spawn only onto keys occupied in N(s); 0 = off."""
        _check(lib().orc_set_initiator(self._ctx, int(min_walkers)), "set_initiator")

    def set_integrator(self, integrator):
        """'euler' or 'ab2' (clears N(s-1))."""
        _check(lib().orc_set_integrator(self._ctx, {"euler": 0, "ab2": 1}[integrator]),
               "integrator")

    def set_proposal(self, kind, k=1, mlp=None):
        """Spawn proposal (reading R18): kind 'comb' (default), 'uniform', 'heatbath' or 'mlp'
        with k samples per parent; mlp = (w1 int8 [32, 64], b1 int32 [32], w2 int8 [64, 32],
        b2 int32 [64], s1)."""
        kinds = {"comb": 0, "uniform": 1, "heatbath": 2, "mlp": 3}
        kd = kinds[kind]
        args = [None, None, None, None, 0]
        if kd == 3:
            w1, b1, w2, b2, s1 = mlp
            self._mlp = (np.ascontiguousarray(w1, dtype=np.int8),
                         np.ascontiguousarray(b1, dtype=np.int32),
                         np.ascontiguousarray(w2, dtype=np.int8),
                         np.ascontiguousarray(b2, dtype=np.int32))
            assert self._mlp[0].shape == (MLP_HIDDEN, MLP_IN)
            assert self._mlp[2].shape == (MLP_OUT, MLP_HIDDEN)
            args = [_p(self._mlp[0], ctypes.c_int8), _p(self._mlp[1], ctypes.c_int32),
                    _p(self._mlp[2], ctypes.c_int8), _p(self._mlp[3], ctypes.c_int32), int(s1)]
        _check(lib().orc_set_proposal(self._ctx, kd, int(k) if kd else 0, *args), "set_proposal")

    def set_proposal_deep(self, k, net):
        """Proposal kind 4 (reading R21) with k samples per parent; net = (w1 int8 [128, 128],
        b1 int32 [128], w2 int8 [128, 128], b2 int32 [128], w3 int8 [64, 128], b3 int32 [64],
        s1, s2)."""
        w1, b1, w2, b2, w3, b3, s1, s2 = net
        arr = [np.ascontiguousarray(w1, dtype=np.int8), np.ascontiguousarray(b1, dtype=np.int32),
               np.ascontiguousarray(w2, dtype=np.int8), np.ascontiguousarray(b2, dtype=np.int32),
               np.ascontiguousarray(w3, dtype=np.int8), np.ascontiguousarray(b3, dtype=np.int32)]
        assert arr[0].shape == (DEEP_HIDDEN, DEEP_IN) and arr[2].shape == (DEEP_HIDDEN, DEEP_HIDDEN)
        assert arr[4].shape == (DEEP_OUT, DEEP_HIDDEN)
        self._deep = arr
        ct = [ctypes.c_int8, ctypes.c_int32] * 3
        _check(lib().orc_set_proposal_deep(self._ctx, int(k),
                                           *[_p(a, t) for a, t in zip(arr, ct)], int(s1), int(s2)),
               "set_proposal_deep")

    def deep_scores(self, key, active):
        """Kind 4 scores of one key with the weight-channel indicator bits `active` (an int < 2^128:
        bit m set where channel m is nonzero)."""
        act = np.array([active & ((1 << 64) - 1), active >> 64], dtype=np.uint64)
        out = np.zeros(DEEP_OUT, dtype=np.int32)
        _check(lib().orc_deep_scores(self._ctx, int(key), _p(act, ctypes.c_uint64),
                                     _p(out, ctypes.c_int32)), "deep_scores")
        return out

    def step_active(self, s, gamma):
        """The step's weight-channel indicator bits (an int < 2^128) for weight rows s, gamma."""
        s = np.ascontiguousarray(np.asarray(s, dtype=np.float64).reshape(-1) if self.n_h
                                 else np.zeros(1))
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(-1) if self.n_l
                                 else np.zeros(1))
        out = np.zeros(2, dtype=np.uint64)
        _check(lib().orc_step_active(self._ctx, _p(s, ctypes.c_double), _p(g, ctypes.c_double),
                                     _p(out, ctypes.c_uint64)), "step_active")
        return int(out[0]) | (int(out[1]) << 64)

    def mlp_scores(self, key):
        out = np.zeros(MLP_OUT, dtype=np.int32)
        _check(lib().orc_mlp_scores(self._ctx, int(key), _p(out, ctypes.c_int32)), "mlp_scores")
        return out

    def counters(self):
        w, k, ch, mx = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        lib().orc_counters(self._ctx, ctypes.byref(w), ctypes.byref(k), ctypes.byref(ch),
                           ctypes.byref(mx))
        return dict(walker_steps=w.value, key_steps=k.value, child_steps=ch.value,
                    max_children=mx.value)

    @property
    def step_index(self):
        return lib().orc_get_step(self._ctx)

    def export(self, replica):
        m = lib().orc_size(self._ctx, int(replica))
        k = np.zeros(max(m, 1), np.uint64); a = np.zeros(max(m, 1), np.int32)
        b = np.zeros(max(m, 1), np.int32); n = ctypes.c_uint64()
        _check(lib().orc_export(self._ctx, int(replica), _p(k, ctypes.c_uint64),
                                _p(a, ctypes.c_int32), _p(b, ctypes.c_int32), m,
                                ctypes.byref(n)), "export")
        return k[:m].copy(), a[:m].copy(), b[:m].copy()

    def import_(self, replica, keys, re, im, step):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        re = np.ascontiguousarray(re, dtype=np.int32)
        im = np.ascontiguousarray(im, dtype=np.int32)
        _check(lib().orc_import(self._ctx, int(replica), _p(keys, ctypes.c_uint64),
                                _p(re, ctypes.c_int32), _p(im, ctypes.c_int32), len(keys),
                                int(step)), "import")

    def set_prev(self, replica, keys, re, im, s_prev, gamma_prev):
        """AB2: N(s-1) of one replica and the weights of step s-1."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        re = np.ascontiguousarray(re, dtype=np.int32)
        im = np.ascontiguousarray(im, dtype=np.int32)
        s, g = self._w(s_prev, gamma_prev)
        _check(lib().orc_set_prev(self._ctx, int(replica), _p(keys, ctypes.c_uint64),
                                  _p(re, ctypes.c_int32), _p(im, ctypes.c_int32), len(keys),
                                  _p(s, ctypes.c_double), _p(g, ctypes.c_double)), "set_prev")

    def export_prev(self, replica):
        """AB2: N(s-1) of one replica."""
        n = ctypes.c_uint64()
        lib().orc_export_prev(self._ctx, int(replica), None, None, None, 0, ctypes.byref(n))
        m = n.value
        k = np.zeros(max(m, 1), np.uint64); a = np.zeros(max(m, 1), np.int32)
        b = np.zeros(max(m, 1), np.int32)
        _check(lib().orc_export_prev(self._ctx, int(replica), _p(k, ctypes.c_uint64),
                                     _p(a, ctypes.c_int32), _p(b, ctypes.c_int32), m,
                                     ctypes.byref(n)), "export_prev")
        return k[:m].copy(), a[:m].copy(), b[:m].copy()

    def observe(self, replica, pauli=(), lookup=()):
        px = np.ascontiguousarray([p[0] for p in pauli] or [0], dtype=np.uint64)
        pz = np.ascontiguousarray([p[1] for p in pauli] or [0], dtype=np.uint64)
        lk = np.ascontiguousarray(list(lookup) or [0], dtype=np.uint64)
        npl, nlk = len(pauli), len(lookup)
        n_occ = ctypes.c_uint64(); n_tot = ctypes.c_uint64()
        nd = np.zeros(2, np.int64); pv = np.zeros((max(npl, 1), 2), np.int64)
        lv = np.zeros((max(nlk, 1), 2), np.int64); e2 = np.zeros(2, np.uint64)
        _check(lib().orc_observe(self._ctx, int(replica), npl, _p(px, ctypes.c_uint64),
                                 _p(pz, ctypes.c_uint64), nlk, _p(lk, ctypes.c_uint64),
                                 ctypes.byref(n_occ), ctypes.byref(n_tot),
                                 _p(nd, ctypes.c_int64), _p(pv, ctypes.c_int64),
                                 _p(lv, ctypes.c_int64), _p(e2, ctypes.c_uint64)), "observe")
        return dict(n_occ=n_occ.value, n_tot=n_tot.value, ndiag=complex(nd[0], nd[1]),
                    ndiag_int=(int(nd[0]), int(nd[1])), pauli=pv[:npl].copy(),
                    lookup=lv[:nlk].copy(), eps2=int(e2[0]) + (int(e2[1]) << 64))
