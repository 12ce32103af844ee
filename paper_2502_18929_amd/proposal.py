"""Training of the spawn-proposal MLP on statistics of the method's own runs.

The proposal (C ABI qmc_set_proposal, kind 3) draws a parent's channels with probabilities from
integer scores of an int8 MLP of the key bits.  Its ideal target is the heat-bath choice of the
End Matter's spawn step: a channel's probability proportional to |L| of that column entry.  The
statistics come from the library itself: a plain run of the workload, the keys its walkers
occupy at a few steps, and at each such key the magnitude |Re c_g| + |Im c_g| of every
off-diagonal column group's Q32 coefficient under that step's quantized table (the per-walker
spawn amount of the group).  A float MLP with the network's shape is fitted to these targets
(mean squared error, Adam) and then quantized to the ABI's integers: w1 int8 [32, 64],
b1 int32 [32], the hidden shift, w2 int8 [64, 32], b2 int32 [64].  Scores are only compared with
each other, so the overall scale of the quantized network is free.
"""
import numpy as np

from . import binding

N_IN, N_HIDDEN, N_OUT = 64, 32, 64


def features(keys, nbits):
    """Network input of each key: +1 where bit b is set, -1 where clear (b < nbits), 0 past."""
    keys = np.asarray(keys, dtype=np.uint64)
    b = np.arange(N_IN, dtype=np.uint64)
    bits = ((keys[:, None] >> np.minimum(b, 63)[None, :]) & np.uint64(1)).astype(np.int64)
    x = 2 * bits - 1
    x[:, b >= nbits] = 0
    return x


def group_magnitudes(table, keys):
    """|Re c_g(key)| + |Im c_g(key)| of the off-diagonal groups g = 1.. of a quantized table, for
    every key: c_g = sum over the group's terms of (-1)^popcount(zmask & key) q."""
    keys = np.asarray(keys, dtype=np.uint64)
    gs = table["gstart"].astype(np.int64)
    G = len(table["gxmask"])
    out = np.zeros((len(keys), max(G - 1, 0)), dtype=np.float64)
    for g in range(1, G):
        cre = np.zeros(len(keys), dtype=np.int64)
        cim = np.zeros(len(keys), dtype=np.int64)
        for t in range(gs[g], gs[g + 1]):
            par = np.bitwise_count(keys & np.uint64(table["zmask"][t])) & 1
            sgn = 1 - 2 * par.astype(np.int64)
            cre += sgn * int(table["q"][t, 0])
            cim += sgn * int(table["q"][t, 1])
        out[:, g - 1] = np.abs(cre) + np.abs(cim)
    return out


def spawn_statistics(ctx, w, stop, at, replica=0):
    """Run the plain step of workload `w` on context `ctx` from its current state up to `stop`
    and collect (keys, targets) at the steps in `at`: the occupied keys of one replica and the
    per-group magnitudes of that step's table there (first N_OUT groups, zero-padded)."""
    keys_all, tgt_all = [], []
    s0 = ctx.counters()["step"]
    for a in sorted(at):
        if a > s0:
            ctx.run_workload(w, s0, a)
            s0 = a
        k, _, _ = ctx.export(replica)
        if len(k) == 0:
            continue
        tab = binding.coeff_table(w.n, w.dt, w.h, w.lops, w.s[a], w.gamma[a])
        m = group_magnitudes(tab, k)[:, :N_OUT]
        t = np.zeros((len(k), N_OUT))
        t[:, :m.shape[1]] = m
        keys_all.append(k)
        tgt_all.append(t)
    if s0 < stop:
        ctx.run_workload(w, s0, stop)
    return np.concatenate(keys_all), np.concatenate(tgt_all)


def fit(keys, targets, nbits, iters=400, lr=3e-3, batch=2048, seed=0):
    """Float MLP (N_IN -> N_HIDDEN relu -> N_OUT) fitted to targets scaled to [0, 1]."""
    rng = np.random.default_rng(seed)
    X = features(keys, nbits).astype(np.float64)
    Y = targets / max(float(targets.max()), 1e-300)
    params = [rng.normal(0, 1 / np.sqrt(max(nbits, 1)), (N_HIDDEN, N_IN)), np.zeros(N_HIDDEN),
              rng.normal(0, 1 / np.sqrt(N_HIDDEN), (N_OUT, N_HIDDEN)), np.full(N_OUT, Y.mean())]
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    for it in range(1, iters + 1):
        idx = rng.integers(0, len(X), size=min(batch, len(X)))
        x, y = X[idx], Y[idx]
        W1, b1, W2, b2 = params
        a = x @ W1.T + b1
        h = np.maximum(a, 0)
        out = h @ W2.T + b2
        d = 2 * (out - y) / len(x)
        gW2, gb2 = d.T @ h, d.sum(0)
        dh = (d @ W2) * (a > 0)
        gW1, gb1 = dh.T @ x, dh.sum(0)
        for i, gr in enumerate([gW1, gb1, gW2, gb2]):
            m[i] = 0.9 * m[i] + 0.1 * gr
            v[i] = 0.999 * v[i] + 0.001 * gr * gr
            params[i] -= lr * (m[i] / (1 - 0.9 ** it)) / (np.sqrt(v[i] / (1 - 0.999 ** it)) + 1e-8)
    return params


def quantize(params, keys, nbits):
    """Integer network of the ABI from the float one: w1 / b1 in units of max|w1| / 127, the
    hidden shift that keeps the largest hidden value of the training keys near 127, w2 in units
    of max|w2| / 127 and b2 in the matching unit of the output."""
    W1, b1, W2, b2 = params
    s_1 = max(np.abs(W1).max(), 1e-12) / 127.0
    w1q = np.clip(np.rint(W1 / s_1), -127, 127).astype(np.int8)
    b1q = np.rint(b1 / s_1).astype(np.int64)
    a = features(keys, nbits) @ w1q.T.astype(np.int64) + b1q
    amax = max(int(a.max()), 1)
    shift = int(max(0, int(np.ceil(np.log2(amax / 127.0))))) if amax > 127 else 0
    s_2 = max(np.abs(W2).max(), 1e-12) / 127.0
    w2q = np.clip(np.rint(W2 / s_2), -127, 127).astype(np.int8)
    unit = s_2 * s_1 * (1 << shift)      # one output count in float units
    b2q = np.clip(np.rint(b2 / unit), -(1 << 24), 1 << 24).astype(np.int32)
    return (w1q, np.clip(b1q, -(1 << 30), 1 << 30).astype(np.int32), w2q, b2q, shift)


def scores(mlp, keys, nbits):
    """Integer scores of the quantized network (the ABI's definition), for inspection."""
    w1, b1, w2, b2, s1 = mlp
    a = features(keys, nbits) @ w1.T.astype(np.int64) + b1
    h = np.minimum(np.where(a > 0, a, 0) >> s1, 127)
    return h @ w2.T.astype(np.int64) + b2


def train(ctx, w, stop, at, seed=0):
    """Statistics from a plain run of `w` on `ctx` (advanced to `stop`), then fit and quantize.
    Returns the MLP tuple for QMC.set_proposal('mlp', ...) and the fit's correlation between
    the integer scores and the targets on the training keys."""
    keys, tgt = spawn_statistics(ctx, w, stop, at)
    nbits = 2 * w.n
    params = fit(keys, tgt, nbits, seed=seed)
    mlp = quantize(params, keys, nbits)
    sc = scores(mlp, keys, nbits)[:, :tgt.shape[1]].astype(np.float64).ravel()
    tv = tgt.ravel()
    corr = float(np.corrcoef(sc, tv)[0, 1]) if sc.std() > 0 and tv.std() > 0 else 0.0
    return mlp, corr
