"""ctypes binding of libqmc (include/qmc.h): argument marshalling only.

Every step of the population dynamics runs in the HIP kernels of ``csrc/``; PyTorch provides
the device workspace (a uint8 tensor) and the stream.  There is no CPU fallback: without the
built library or without a GPU, construction raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqmc.so")

QMC_OK = 0
QMC_ERR_ARG = -1
QMC_ERR_DT = -2
QMC_ERR_STORE_CAP = -3
QMC_ERR_SPAWN_CAP = -4
QMC_ERR_COUNT_OVERFLOW = -5
QMC_ERR_HIP = -6
QMC_ERR_STATE = -8

EXPORTED = ["qmc_workspace_bytes", "qmc_init", "qmc_step", "qmc_step_path",
            "qmc_set_integrator", "qmc_set_prev", "qmc_export_prev", "qmc_pulse",
            "qmc_set_shift", "qmc_set_initiator", "qmc_set_proposal", "qmc_tune_sort",
            "qmc_use_graphs", "qmc_observe",
            "qmc_export", "qmc_import", "qmc_counters",
            "qmc_profile", "qmc_profile_read", "qmc_profile_read_class", "qmc_coeff_table",
            "qmc_last_error",
            "qmc_destroy", "qmc_workspace_bytes_batch", "qmc_init_batch", "qmc_pulse_batch",
            "qmc_observe_noalloc", "qmc_small_limit", "qmc_set_proposal_deep", "qmc_log_spawns"]


class Monomial(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint64), ("z", ctypes.c_uint64),
                ("re", ctypes.c_double), ("im", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_uint32), ("n_replicas", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("dt", ctypes.c_double),
                ("walker_target", ctypes.c_uint64), ("store_capacity", ctypes.c_uint64),
                ("spawn_capacity", ctypes.c_uint64), ("shift_mode", ctypes.c_uint32),
                ("shift_zeta", ctypes.c_double), ("shift_period", ctypes.c_uint32),
                ("shift_target", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("step", ctypes.c_uint32), ("n_occ_total", ctypes.c_uint64),
                ("walker_steps", ctypes.c_uint64), ("key_steps", ctypes.c_uint64),
                ("child_steps", ctypes.c_uint64), ("out_steps", ctypes.c_uint64),
                ("rebalances", ctypes.c_uint64), ("spawn_steps", ctypes.c_uint64)]


class Model(ctypes.Structure):
    _fields_ = [("n_h", ctypes.c_uint32), ("h", ctypes.POINTER(Monomial)),
                ("n_l", ctypes.c_uint32), ("l_off", ctypes.POINTER(ctypes.c_uint32)),
                ("l", ctypes.POINTER(Monomial))]


class ObsSpec(ctypes.Structure):
    _fields_ = [("n_pauli", ctypes.c_uint32), ("px", ctypes.POINTER(ctypes.c_uint64)),
                ("pz", ctypes.POINTER(ctypes.c_uint64)), ("n_psi", ctypes.c_uint32),
                ("psi_index", ctypes.POINTER(ctypes.c_uint64)),
                ("psi_re", ctypes.POINTER(ctypes.c_double)),
                ("psi_im", ctypes.POINTER(ctypes.c_double)), ("want_eps", ctypes.c_uint32)]


P64 = ctypes.POINTER(ctypes.c_uint64)
PI64 = ctypes.POINTER(ctypes.c_int64)
PD = ctypes.POINTER(ctypes.c_double)


class ObsOut(ctypes.Structure):
    _fields_ = [("n_occ", P64), ("n_tot", P64), ("ndiag", PI64), ("pauli", PI64), ("eps2", P64),
                ("trace", PD), ("theta", PD), ("pauli_val", PD), ("fidelity", PD), ("eps", PD),
                ("shift", PD)]


_lib = None


def lib():
    """Load libqmc.so (built by ``paper_2502_18929_amd.build``); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        u32, u64, i32, dbl, vp = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_void_p)
        P = ctypes.POINTER
        L.qmc_workspace_bytes.argtypes = [P(Config), P(Model), P(ctypes.c_size_t)]
        L.qmc_init.argtypes = [P(Config), P(Model), P(u64), P(i32), P(i32), u64, vp,
                               ctypes.c_size_t, vp, P(vp)]
        L.qmc_step.argtypes = [vp, u32, P(dbl), P(dbl)]
        L.qmc_pulse.argtypes = [vp, u64, u64]
        L.qmc_pulse_batch.argtypes = [vp, P(u64), P(u64)]
        L.qmc_workspace_bytes_batch.argtypes = [P(Config), u32, P(Model), P(ctypes.c_size_t)]
        L.qmc_init_batch.argtypes = [P(Config), u32, P(Model), P(P(u64)), P(P(i32)), P(P(i32)),
                                     P(u64), vp, ctypes.c_size_t, vp, P(vp)]
        L.qmc_set_shift.argtypes = [vp, u32, dbl]
        L.qmc_set_initiator.argtypes = [vp, ctypes.c_uint64]
        i8p = P(ctypes.c_int8)
        L.qmc_set_proposal.argtypes = [vp, i32, u32, i8p, P(i32), i8p, P(i32), u32]
        L.qmc_set_proposal_deep.argtypes = [vp, u32, i8p, P(i32), i8p, P(i32), i8p, P(i32), u32,
                                            u32]
        L.qmc_log_spawns.argtypes = [vp, vp, u64, vp]
        L.qmc_tune_sort.argtypes = [vp, u32, P(u32)]
        L.qmc_use_graphs.argtypes = [vp, i32]
        L.qmc_observe.argtypes = [vp, P(ObsSpec), P(ObsOut)]
        L.qmc_export.argtypes = [vp, u32, P(u64), P(i32), P(i32), u64, P(u64)]
        L.qmc_import.argtypes = [vp, u32, P(u64), P(i32), P(i32), u64, u32]
        L.qmc_counters.argtypes = [vp, P(Stats)]
        L.qmc_profile.argtypes = [vp, ctypes.c_int32]
        L.qmc_step_path.argtypes = [vp, ctypes.c_int32]
        L.qmc_small_limit.argtypes = [vp, u32]
        L.qmc_set_integrator.argtypes = [vp, ctypes.c_int32]
        L.qmc_set_prev.argtypes = [vp, u32, P(u64), P(i32), P(i32), u64, P(dbl), P(dbl)]
        L.qmc_export_prev.argtypes = [vp, u32, P(u64), P(i32), P(i32), u64, P(u64)]
        L.qmc_profile_read.argtypes = [vp, P(dbl), P(u64), P(Stats)]
        L.qmc_profile_read_class.argtypes = [vp, ctypes.c_int32, P(dbl), P(u64), P(Stats)]
        L.qmc_coeff_table.argtypes = [P(Config), P(Model), P(dbl), P(dbl), dbl, u32, u32, P(u32),
                                      P(u64), P(u32), P(u32), P(u64), P(ctypes.c_int64)]
        L.qmc_last_error.argtypes = [vp]
        L.qmc_last_error.restype = ctypes.c_char_p
        L.qmc_destroy.argtypes = [vp]
        L.qmc_destroy.restype = None
        L.qmc_observe_noalloc.argtypes = [u32, u32, vp, vp, u64, P(ctypes.c_int64), P(ObsSpec),
                                          P(ObsOut), vp]
        _lib = L
    return _lib


class QMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libqmc error {code}: {msg}")
        self.code = code


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _monos(lst):
    arr = (Monomial * max(1, len(lst)))()
    for i, (x, z, c) in enumerate(lst):
        c = complex(c)
        arr[i] = Monomial(int(x), int(z), c.real, c.imag)
    return arr


class QMC:
    """One libqmc context: R replicas of one model (or of each model of a batch of circuits,
    see ``QMC.batch``), advanced on one HIP stream."""

    _integrator = "euler"  # the context's default time integrator

    def __init__(self, n, n_replicas, seed, dt, h, lops, keys, re, im, store_capacity,
                 spawn_capacity, walker_target=0, stream=None, shift=None):
        """shift = None (constant shift, 0 unless set_shift) or a dict of the variable-shift
        control: {"zeta": ..., "period": A, "target": N^tot at which it starts}."""
        self._setup(n, n_replicas, seed, dt, [(h, lops, keys, re, im)], store_capacity,
                    spawn_capacity, walker_target, stream, shift)

    @classmethod
    def batch(cls, n, n_replicas, seed, dt, circuits, store_capacity, spawn_capacity,
              stream=None, shift=None):
        """A batch of circuits on n qubits: circuits = [(h, lops, keys, re, im), ...] (a
        smaller circuit uses only its low qubits).  Replica r of circuit c is segment
        c * n_replicas + r for export/import/observe/set_shift; step() takes the weights of all
        circuits side by side (circuit 0's columns first)."""
        self = cls.__new__(cls)
        self._setup(n, n_replicas, seed, dt, circuits, store_capacity, spawn_capacity, 0, stream,
                    shift)
        return self

    def _setup(self, n, n_replicas, seed, dt, circuits, store_capacity, spawn_capacity,
               walker_target, stream, shift=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libqmc needs a HIP device; none is visible")
        L = lib()
        C = len(circuits)
        self.n, self.C, self.Rc = int(n), C, int(n_replicas)
        self.R = C * self.Rc
        self.n_h = sum(len(c[0]) for c in circuits)
        self.n_l = sum(len(c[1]) for c in circuits)
        self._keep = []
        models = (Model * C)()
        keys_p = (P64 * C)()
        re_p = (ctypes.POINTER(ctypes.c_int32) * C)()
        im_p = (ctypes.POINTER(ctypes.c_int32) * C)()
        n0 = np.zeros(C, dtype=np.uint64)
        for ci, (h, lops, keys, re, im) in enumerate(circuits):
            hm = _monos(h)
            lm = _monos([m for op in lops for m in op])
            off = np.zeros(len(lops) + 1, dtype=np.uint32)
            for kk, op in enumerate(lops):
                off[kk + 1] = off[kk] + len(op)
            keys = np.ascontiguousarray(keys, dtype=np.uint64)
            re = np.ascontiguousarray(re, dtype=np.int32)
            im = np.ascontiguousarray(im, dtype=np.int32)
            self._keep += [hm, lm, off, keys, re, im]
            models[ci] = Model(len(h), hm, len(lops), _ptr(off, ctypes.c_uint32), lm)
            keys_p[ci] = _ptr(keys, ctypes.c_uint64)
            re_p[ci] = _ptr(re, ctypes.c_int32)
            im_p[ci] = _ptr(im, ctypes.c_int32)
            n0[ci] = len(keys)
        self._models, self._n0 = models, n0
        sh = shift or {}
        self._cfg = Config(self.n, self.Rc, int(seed), float(dt), int(walker_target),
                           int(store_capacity), int(spawn_capacity), 1 if shift else 0,
                           float(sh.get("zeta", 0.0)), int(sh.get("period", 1)),
                           int(sh.get("target", 0)))
        nb = ctypes.c_size_t()
        rc = L.qmc_workspace_bytes_batch(ctypes.byref(self._cfg), C, models, ctypes.byref(nb))
        if rc:
            raise QMCError(rc, "invalid configuration")
        self.ws_bytes = nb.value
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._ctx = ctypes.c_void_p()
        rc = L.qmc_init_batch(ctypes.byref(self._cfg), C, models, keys_p, re_p, im_p,
                              _ptr(n0, ctypes.c_uint64), ctypes.c_void_p(aligned),
                              self.ws_bytes, ctypes.c_void_p(stream.cuda_stream),
                              ctypes.byref(self._ctx))
        if rc:
            raise QMCError(rc, "qmc_init failed")

    @classmethod
    def from_workload(cls, w, store_capacity=None, spawn_capacity=None, n_replicas=None,
                      seed=None, shift=None):
        R = w.n_replicas if n_replicas is None else n_replicas
        if store_capacity is None:
            store_capacity = min(1 << (2 * w.n), 1 << 20)
        if spawn_capacity is None:
            spawn_capacity = store_capacity
        return cls(w.n, R, w.seed if seed is None else seed, w.dt, w.h, w.lops, w.init_keys,
                   w.init_re, w.init_im, store_capacity, spawn_capacity,
                   walker_target=w.walker_target, shift=shift)

    def _check(self, rc):
        if rc:
            msg = lib().qmc_last_error(self._ctx)
            raise QMCError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_ctx", None):
            lib().qmc_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()
        self._ws = None  # the device workspace goes back to torch's allocator now

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, s, gamma):
        """s: [nsteps, n_h] weights, gamma: [nsteps, n_l] rates."""
        s = np.asarray(s, dtype=np.float64)
        g = np.asarray(gamma, dtype=np.float64)
        nsteps = s.shape[0] if s.ndim == 2 else g.shape[0]
        s = np.ascontiguousarray(s.reshape(nsteps, self.n_h) if self.n_h else np.zeros((nsteps, 1)))
        g = np.ascontiguousarray(g.reshape(nsteps, self.n_l) if self.n_l else np.zeros((nsteps, 1)))
        self._check(lib().qmc_step(self._ctx, nsteps, _ptr(s, ctypes.c_double),
                                   _ptr(g, ctypes.c_double)))

    def run_workload(self, w, start=0, stop=None):
        """Advance through steps [start, stop) of a workload, applying its ideal pulses.  A
        workload whose steps differ in length (finite pulses sub-stepped) needs the Euler step:
        AB2's weights 3/2 and -1/2 assume a uniform step."""
        stop = w.nsteps if stop is None else stop
        sdt = getattr(w, "step_dt", None)
        if (self._integrator == "ab2" and sdt is not None and
                not np.all(sdt[start:stop] == sdt[start])):
            raise QMCError(QMC_ERR_ARG, "AB2 needs a uniform step; this workload sub-steps "
                                        "its pulses (use the Euler step)")
        for a, b, pulses in w.segments():
            if b <= start or a >= stop:
                continue
            if a >= start:
                for (px, pz) in pulses:
                    self.pulse(px, pz)
            lo, hi = max(a, start), min(b, stop)
            self.step(w.s[lo:hi], w.gamma[lo:hi])
        if stop == w.nsteps:
            for (px, pz) in w.pulses.get(w.nsteps, []):
                self.pulse(px, pz)

    def run_batch_workload(self, bw, start=0, stop=None):
        """Advance a batch context through steps [start, stop) of a BatchWorkload, applying the
        circuits' pulses."""
        stop = bw.nsteps if stop is None else stop
        for a, b, masks in bw.segments():
            if b <= start or a >= stop:
                continue
            if a >= start and masks is not None:
                self.pulse_batch(*masks)
            lo, hi = max(a, start), min(b, stop)
            self.step(*bw.weights(lo, hi))

    def pulse(self, x, z):
        self._check(lib().qmc_pulse(self._ctx, int(x), int(z)))

    def pulse_batch(self, xs, zs):
        """Circuit c of a batch takes the Pauli X^xs[c] Z^zs[c]."""
        x = np.ascontiguousarray(xs, dtype=np.uint64)
        z = np.ascontiguousarray(zs, dtype=np.uint64)
        assert len(x) == self.C and len(z) == self.C
        self._check(lib().qmc_pulse_batch(self._ctx, _ptr(x, ctypes.c_uint64),
                                          _ptr(z, ctypes.c_uint64)))

    def set_shift(self, replica, shift):
        self._check(lib().qmc_set_shift(self._ctx, int(replica), float(shift)))

    def set_initiator(self, min_walkers):
        """Initiator approximation: parents with |re| + |im| < min_walkers spawn only onto keys
        occupied in N(s); 0 = off.  initiator_threshold(xi, n_diag) gives ceil(xi * N^diag)."""
        self._check(lib().qmc_set_initiator(self._ctx, int(min_walkers)))

    def use_graphs(self, on=True):
        """Capture each chunk of streamed steps into a HIP graph and replay it."""
        self._check(lib().qmc_use_graphs(self._ctx, 1 if on else 0))

    def tune_sort(self, records_per_thread=0):
        """Tile size of the look-back sort that re-sorts the store after a pulse with x flips
        (the per-step sort has its own): 0 autotunes (times 8, 12, 16, 24 records per thread and
        keeps the fastest), else sets it.  Returns the size in use."""
        out = ctypes.c_uint32()
        self._check(lib().qmc_tune_sort(self._ctx, int(records_per_thread), ctypes.byref(out)))
        return int(out.value)

    PROPOSALS = {"comb": 0, "uniform": 1, "heatbath": 2, "mlp": 3}

    def set_proposal(self, kind, samples=1, mlp=None):
        """Spawn proposal: 'comb' (the plain step), 'uniform', 'heatbath' or 'mlp' with `samples`
        channel draws per parent; mlp = (w1 int8 [32, 64], b1 int32 [32], w2 int8 [64, 32],
        b2 int32 [64], hidden_shift)."""
        kd = self.PROPOSALS[kind]
        if kd == 3:
            w1, b1, w2, b2, s1 = mlp
            arrs = [np.ascontiguousarray(w1, dtype=np.int8), np.ascontiguousarray(b1, dtype=np.int32),
                    np.ascontiguousarray(w2, dtype=np.int8), np.ascontiguousarray(b2, dtype=np.int32)]
            if arrs[0].shape != (32, 64) or arrs[1].shape != (32,) or arrs[2].shape != (64, 32) \
                    or arrs[3].shape != (64,):
                raise ValueError("MLP shapes: w1 [32, 64], b1 [32], w2 [64, 32], b2 [64]")
            self._check(lib().qmc_set_proposal(
                self._ctx, kd, int(samples), _ptr(arrs[0], ctypes.c_int8), _ptr(arrs[1], ctypes.c_int32),
                _ptr(arrs[2], ctypes.c_int8), _ptr(arrs[3], ctypes.c_int32), int(s1)))
        else:
            self._check(lib().qmc_set_proposal(self._ctx, kd, int(samples) if kd else 0, None, None,
                                               None, None, 0))

    def log_spawns(self, capacity):
        """Start logging the plain comb's off-diagonal spawn events of the streamed path into a
        device buffer of `capacity` events (the path is set to 'streamed'); log_read() returns
        them.  capacity = 0 stops logging."""
        import torch
        if capacity <= 0:
            self._check(lib().qmc_log_spawns(self._ctx, None, 0, None))
            self._log = None
            return
        ev = torch.empty(int(capacity) * 24, dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        self._log = (ev, cnt, int(capacity))
        self.set_path("streamed")
        self._check(lib().qmc_log_spawns(self._ctx, ctypes.c_void_p(ev.data_ptr()), int(capacity),
                                         ctypes.c_void_p(cnt.data_ptr())))

    def log_read(self):
        """(events, total): the logged events as a numpy structured array (key, step, group, re,
        im) and the number drawn (more than stored when the buffer filled up)."""
        import torch
        ev, cnt, cap = self._log
        torch.cuda.synchronize()
        total = int(cnt.item())
        n = min(total, cap)
        dt = np.dtype([("key", "<u8"), ("step", "<u4"), ("group", "<u4"), ("re", "<i4"),
                       ("im", "<i4")])
        raw = ev[:n * 24].cpu().numpy()
        return raw.view(dt).copy(), total

    def set_proposal_deep(self, samples, net):
        """Spawn proposal kind 4 (the deeper int8 network of the key bits and the step's active
        weight channels): net = (w1 int8 [128, 128], b1 int32 [128], w2 int8 [128, 128],
        b2 int32 [128], w3 int8 [64, 128], b3 int32 [64], shift1, shift2)."""
        w1, b1, w2, b2, w3, b3, s1, s2 = net
        shapes = [(128, 128), (128,), (128, 128), (128,), (64, 128), (64,)]
        types = [np.int8, np.int32] * 3
        arrs = [np.ascontiguousarray(a, dtype=t) for a, t in zip((w1, b1, w2, b2, w3, b3), types)]
        if [a.shape for a in arrs] != shapes:
            raise ValueError("network shapes: w1 [128, 128], b1 [128], w2 [128, 128], b2 [128], "
                             "w3 [64, 128], b3 [64]")
        ct = [ctypes.c_int8, ctypes.c_int32] * 3
        self._check(lib().qmc_set_proposal_deep(self._ctx, int(samples),
                                                *[_ptr(a, t) for a, t in zip(arrs, ct)],
                                                int(s1), int(s2)))

    def observe(self, pauli=(), psi=(), want_eps=False):
        spec, o, out, keep = _obs_args(self.R, pauli, psi, want_eps)
        self._check(lib().qmc_observe(self._ctx, ctypes.byref(spec), ctypes.byref(out)))
        return _obs_result(o, len(pauli))

    def export(self, replica):
        n = ctypes.c_uint64()
        cap = 0
        rc = lib().qmc_export(self._ctx, int(replica), None, None, None, cap, ctypes.byref(n))
        if rc not in (QMC_OK, QMC_ERR_ARG):
            self._check(rc)
        m = n.value
        k = np.zeros(max(m, 1), np.uint64)
        a = np.zeros(max(m, 1), np.int32)
        b = np.zeros(max(m, 1), np.int32)
        self._check(lib().qmc_export(self._ctx, int(replica), _ptr(k, ctypes.c_uint64),
                                     _ptr(a, ctypes.c_int32), _ptr(b, ctypes.c_int32), m,
                                     ctypes.byref(n)))
        return k[:m].copy(), a[:m].copy(), b[:m].copy()

    def import_(self, replica, keys, re, im, step):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        re = np.ascontiguousarray(re, dtype=np.int32)
        im = np.ascontiguousarray(im, dtype=np.int32)
        self._check(lib().qmc_import(self._ctx, int(replica), _ptr(keys, ctypes.c_uint64),
                                     _ptr(re, ctypes.c_int32), _ptr(im, ctypes.c_int32),
                                     len(keys), int(step)))

    def counters(self):
        st = Stats()
        self._check(lib().qmc_counters(self._ctx, ctypes.byref(st)))
        return dict(step=st.step, n_occ=st.n_occ_total, walker_steps=st.walker_steps,
                    key_steps=st.key_steps, child_steps=st.child_steps, out_steps=st.out_steps,
                    rebalances=st.rebalances, spawn_steps=st.spawn_steps)

    def set_integrator(self, integrator):
        """Time integrator: 'euler' (default) or 'ab2' (clears N(s-1))."""
        self._check(lib().qmc_set_integrator(self._ctx, {"euler": 0, "ab2": 1}[integrator]))
        self._integrator = integrator

    def set_prev(self, replica, keys, re, im, s_prev, gamma_prev):
        """AB2: N(s-1) of one replica and the weights of step s-1."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        re = np.ascontiguousarray(re, dtype=np.int32)
        im = np.ascontiguousarray(im, dtype=np.int32)
        s = np.ascontiguousarray(s_prev if self.n_h else np.zeros(1), dtype=np.float64)
        g = np.ascontiguousarray(gamma_prev if self.n_l else np.zeros(1), dtype=np.float64)
        self._check(lib().qmc_set_prev(self._ctx, int(replica), _ptr(keys, ctypes.c_uint64),
                                       _ptr(re, ctypes.c_int32), _ptr(im, ctypes.c_int32),
                                       len(keys), _ptr(s, ctypes.c_double),
                                       _ptr(g, ctypes.c_double)))

    def export_prev(self, replica):
        """AB2: N(s-1) of one replica (keys ascending)."""
        n = ctypes.c_uint64()
        rc = lib().qmc_export_prev(self._ctx, int(replica), None, None, None, 0, ctypes.byref(n))
        if rc not in (QMC_OK, QMC_ERR_ARG):
            self._check(rc)
        m = n.value
        k = np.zeros(max(m, 1), np.uint64)
        a = np.zeros(max(m, 1), np.int32)
        b = np.zeros(max(m, 1), np.int32)
        self._check(lib().qmc_export_prev(self._ctx, int(replica), _ptr(k, ctypes.c_uint64),
                                          _ptr(a, ctypes.c_int32), _ptr(b, ctypes.c_int32), m,
                                          ctypes.byref(n)))
        return k[:m].copy(), a[:m].copy(), b[:m].copy()

    def set_path(self, path):
        """Step implementation: 'auto' (default), 'fused' (persistent kernel), 'streamed' or
        'small' (the LDS-resident step, while every replica fits)."""
        self._check(lib().qmc_step_path(self._ctx, {"auto": 0, "fused": 1, "streamed": 2,
                                                    "small": 3}[path]))

    def small_limit(self, keys):
        """Keys per replica up to which the automatic path takes the LDS-resident step (0: never;
        at most 1024)."""
        self._check(lib().qmc_small_limit(self._ctx, int(keys)))

    _PROF_CLASSES = {None: -1, "spawn": 0, "sort": 1, "merge": 2, "fused": 3, "small": 4,
                     "step": 5}

    def profile(self, kernel_class):
        """Time one kernel class with HIP events: 'spawn' (the draws of each step's records),
        'sort', 'merge' (streamed path), 'fused' (one persistent launch), 'small' (one
        LDS-resident launch), 'step' (one chunk of whole streamed steps) or None.  'fused' and
        'small' are timed together, each into its own totals (profile_read(kind)); 'step' times
        'merge' beside it."""
        self._check(lib().qmc_profile(self._ctx, self._PROF_CLASSES[kernel_class]))

    def profile_read(self, kernel_class=None):
        """(milliseconds, launches, covered): the timed launches of the profiled class (or of
        `kernel_class`) and the counter sums of the steps they ran (see qmc_profile_read)."""
        ms, n, st = ctypes.c_double(), ctypes.c_uint64(), Stats()
        if kernel_class is None:
            self._check(lib().qmc_profile_read(self._ctx, ctypes.byref(ms), ctypes.byref(n),
                                               ctypes.byref(st)))
        else:
            self._check(lib().qmc_profile_read_class(self._ctx, self._PROF_CLASSES[kernel_class],
                                                     ctypes.byref(ms), ctypes.byref(n),
                                                     ctypes.byref(st)))
        cov = dict(steps=st.step, walker_steps=st.walker_steps, key_steps=st.key_steps,
                   child_steps=st.child_steps, out_steps=st.out_steps,
                   spawn_steps=st.spawn_steps)
        return ms.value, n.value, cov


def _obs_args(R, pauli, psi, want_eps):
    """The qmc_obs_spec and the output arrays of an estimator call over R replicas (the arrays
    are returned too, so they outlive the call)."""
    npl = len(pauli)
    px = np.ascontiguousarray([p[0] for p in pauli] or [0], dtype=np.uint64)
    pz = np.ascontiguousarray([p[1] for p in pauli] or [0], dtype=np.uint64)
    pidx = np.ascontiguousarray([p[0] for p in psi] or [0], dtype=np.uint64)
    pre = np.ascontiguousarray([complex(p[1]).real for p in psi] or [0.0])
    pim = np.ascontiguousarray([complex(p[1]).imag for p in psi] or [0.0])
    spec = ObsSpec(npl, _ptr(px, ctypes.c_uint64), _ptr(pz, ctypes.c_uint64), len(psi),
                   _ptr(pidx, ctypes.c_uint64), _ptr(pre, ctypes.c_double),
                   _ptr(pim, ctypes.c_double), 1 if want_eps else 0)
    o = dict(n_occ=np.zeros(R, np.uint64), n_tot=np.zeros(R, np.uint64),
             ndiag=np.zeros((R, 2), np.int64), pauli=np.zeros((R, max(npl, 1), 2), np.int64),
             eps2=np.zeros((R, 2), np.uint64), trace=np.zeros(R), theta=np.zeros(R),
             pauli_val=np.zeros((R, max(npl, 1), 2)), fidelity=np.zeros((R, 2)),
             eps=np.zeros(R), shift=np.zeros(R))
    out = ObsOut(_ptr(o["n_occ"], ctypes.c_uint64), _ptr(o["n_tot"], ctypes.c_uint64),
                 _ptr(o["ndiag"], ctypes.c_int64), _ptr(o["pauli"], ctypes.c_int64),
                 _ptr(o["eps2"], ctypes.c_uint64), _ptr(o["trace"], ctypes.c_double),
                 _ptr(o["theta"], ctypes.c_double), _ptr(o["pauli_val"], ctypes.c_double),
                 _ptr(o["fidelity"], ctypes.c_double), _ptr(o["eps"], ctypes.c_double),
                 _ptr(o["shift"], ctypes.c_double))
    return spec, o, out, (px, pz, pidx, pre, pim)


def _obs_result(o, npl):
    # a nonzero shift (constant or variable population control) biases the estimators
    o["biased"] = bool(np.any(o["shift"] != 0))
    o["pauli"] = o["pauli"][:, :npl]
    o["pauli_val"] = o["pauli_val"][:, :npl]
    o["eps2_int"] = [int(a) + (int(b) << 64) for a, b in o["eps2"]]
    return o


def observe_noalloc(n, n_replicas, keys, vals, nd0_re, pauli=(), psi=(), want_eps=False,
                    stream=None):
    """qmc_observe_noalloc: the estimators of a sorted store held in device memory, with no
    context and no allocation in the library.  keys: a device tensor of the composite keys
    (replica << 2n | key, ascending; int64 or uint64 storage), vals: a device int32 tensor of
    [len(keys), 2] (re, im); nd0_re: Re N^diag(0) per replica.  Returns what QMC.observe does."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libqmc needs a HIP device; none is visible")
    m = int(keys.numel())
    if vals.dtype != torch.int32 or tuple(vals.shape) != (m, 2) or not vals.is_contiguous():
        raise ValueError("vals must be a contiguous int32 tensor of shape [len(keys), 2]")
    if keys.element_size() != 8 or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous 64-bit tensor")
    nd0 = np.ascontiguousarray(nd0_re, dtype=np.int64)
    if nd0.shape != (int(n_replicas),):
        raise ValueError("nd0_re needs one value per replica")
    spec, o, out, keep = _obs_args(int(n_replicas), pauli, psi, want_eps)
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = lib().qmc_observe_noalloc(int(n), int(n_replicas), ctypes.c_void_p(keys.data_ptr()),
                                   ctypes.c_void_p(vals.data_ptr()), m,
                                   _ptr(nd0, ctypes.c_int64), ctypes.byref(spec),
                                   ctypes.byref(out), ctypes.c_void_p(stream.cuda_stream))
    if rc:
        raise QMCError(rc, "qmc_observe_noalloc failed")
    return _obs_result(o, len(pauli))


def initiator_threshold(xi, n_diag):
    """The initiator threshold in whole walkers for a fraction xi of N^diag (rounded up, exact
    for the decimal fractions used in practice: xi * N^diag computed in integer arithmetic when
    xi is given as a Fraction or a decimal string)."""
    from fractions import Fraction
    x = Fraction(str(xi)) if not isinstance(xi, Fraction) else xi
    v = x * int(n_diag)
    return int(-(-v.numerator // v.denominator))


def coeff_table(n, dt, h, lops, s, gamma, n_replicas=1, scale=1.0):
    """Host-only: the quantized step table the library would use (no device needed), for
    scale * dt * L(t) (1 for Euler; 3/2 and -1/2 for the two AB2 terms)."""
    L = lib()
    hm = _monos(h)
    lm = _monos([m for op in lops for m in op])
    off = np.zeros(len(lops) + 1, dtype=np.uint32)
    for k, op in enumerate(lops):
        off[k + 1] = off[k] + len(op)
    cfg = Config(int(n), int(n_replicas), 0, float(dt), 0, 1, 1, 0, 0.0, 1, 0)
    model = Model(len(h), hm, len(lops), _ptr(off, ctypes.c_uint32), lm)
    s = np.ascontiguousarray(s if len(h) else np.zeros(1), dtype=np.float64)
    g = np.ascontiguousarray(gamma if len(lops) else np.zeros(1), dtype=np.float64)
    cap = 8192
    ng, nt = ctypes.c_uint32(), ctypes.c_uint32()
    gx = np.zeros(cap, np.uint64); gs = np.zeros(cap + 1, np.uint32)
    tz = np.zeros(cap, np.uint64); tq = np.zeros((cap, 2), np.int64)
    rc = L.qmc_coeff_table(ctypes.byref(cfg), ctypes.byref(model), _ptr(s, ctypes.c_double),
                           _ptr(g, ctypes.c_double), float(scale), cap, cap, ctypes.byref(ng),
                           _ptr(gx, ctypes.c_uint64), _ptr(gs, ctypes.c_uint32), ctypes.byref(nt),
                           _ptr(tz, ctypes.c_uint64), _ptr(tq, ctypes.c_int64))
    if rc:
        raise QMCError(rc, "qmc_coeff_table failed")
    G, T = ng.value, nt.value
    return dict(gxmask=gx[:G].copy(), gstart=gs[:G + 1].copy(), zmask=tz[:T].copy(),
                q=tq[:T].copy())
