"""Training of the spawn-proposal networks on statistics of the method's own runs.

The proposal (C ABI qmc_set_proposal, kind 3) draws a parent's channels with probabilities from
integer scores of an int8 MLP of the key bits.  Its ideal target is the heat-bath choice of the
End Matter's spawn step: a channel's probability proportional to |L| of that column entry.  The
statistics come from the library itself: a plain run of the workload with the library's
spawn-event log on, whose off-diagonal events are pooled per parent key into the walkers spawned
into each column group, as fractions of the key's total.  A float MLP with the network's shape
is fitted to these targets (mean squared error, Adam) and then quantized to the ABI's integers:
w1 int8 [32, 64], b1 int32 [32], the hidden shift, w2 int8 [64, 32], b2 int32 [64].  Scores are
only compared with each other, so the overall scale of the quantized network is free.  The
deeper network (kind 4, below) is trained on the same log, pooled per (key, step channels).
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


def pooled_fractions(events, n):
    """Per parent key of logged spawn events (the library's event log), the walkers (|re| + |im|)
    spawned into each of the first N_OUT column groups, as fractions of the key's total over
    those groups; returns (keys, fractions, totals, events per key)."""
    kmask = np.uint64((1 << (2 * n)) - 1) if 2 * n < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    keep = (events["group"] >= 1) & (events["group"] <= N_OUT)
    ev = events[keep]
    key = ev["key"] & kmask
    walkers = np.abs(ev["re"].astype(np.int64)) + np.abs(ev["im"].astype(np.int64))
    uk, inv = np.unique(key, return_inverse=True)
    Y = np.zeros((len(uk), N_OUT))
    np.add.at(Y, (inv, ev["group"].astype(np.int64) - 1), walkers)
    tot = Y.sum(axis=1)
    Y /= np.maximum(tot, 1)[:, None]
    return uk, Y, tot, np.bincount(inv, minlength=len(uk))


def spawn_statistics(ctx, w, stop, capacity=16_000_000):
    """Run the plain step of workload `w` on context `ctx` (streamed, with the library's spawn
    event log) from its current state up to `stop`, and pool the logged events per parent key
    (pooled_fractions): the training keys and targets of the network."""
    ctx.log_spawns(capacity)
    s0 = ctx.counters()["step"]
    if stop > s0:
        ctx.run_workload(w, s0, stop)
    ev, _ = ctx.log_read()
    ctx.log_spawns(0)
    keys, Y, _, nev = pooled_fractions(ev, w.n)
    return keys, Y, nev


def fit(keys, targets, nbits, iters=400, lr=3e-3, batch=2048, seed=0, weights=None):
    """Float MLP (N_IN -> N_HIDDEN relu -> N_OUT) fitted to targets scaled to [0, 1], each key
    drawn into the minibatches in proportion to its weight (default: all alike).  With a key's
    fractions pooled from its spawn events and the weight its number of events, this is the
    least-squares fit over the individual events, whose expectation is the key's spawn
    fractions."""
    rng = np.random.default_rng(seed)
    prob = None
    if weights is not None:
        prob = np.asarray(weights, dtype=np.float64)
        prob = prob / prob.sum()
    X = features(keys, nbits).astype(np.float64)
    Y = targets / max(float(targets.max()), 1e-300)
    params = [rng.normal(0, 1 / np.sqrt(max(nbits, 1)), (N_HIDDEN, N_IN)), np.zeros(N_HIDDEN),
              rng.normal(0, 1 / np.sqrt(N_HIDDEN), (N_OUT, N_HIDDEN)), np.full(N_OUT, Y.mean())]
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    for it in range(1, iters + 1):
        idx = (rng.integers(0, len(X), size=min(batch, len(X))) if prob is None else
               rng.choice(len(X), size=min(batch, len(X)), p=prob))
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


def train(ctx, w, stop, seed=0):
    """Spawn statistics of a plain run of `w` on `ctx` (advanced to `stop`), then fit and
    quantize.  Returns the MLP tuple for QMC.set_proposal('mlp', ...) and the fit's correlation
    between the integer scores and the targets on the training keys."""
    keys, tgt, nev = spawn_statistics(ctx, w, stop)
    nbits = 2 * w.n
    params = fit(keys, tgt, nbits, seed=seed, weights=nev)
    mlp = quantize(params, keys, nbits)
    sc = scores(mlp, keys, nbits)[:, :tgt.shape[1]].astype(np.float64).ravel()
    tv = tgt.ravel()
    corr = float(np.corrcoef(sc, tv)[0, 1]) if sc.std() > 0 and tv.std() > 0 else 0.0
    return mlp, corr


# ---- the deeper network (proposal kind 4) ------------------------------------------------------

DEEP_IN, DEEP_HIDDEN, DEEP_OUT = 128, 128, 64


def active_masks(w):
    """Per step of workload `w`: the bits of its weight channels (H monomials, then Lindblad
    operators) that are nonzero at that step -- the channel inputs of the deeper network."""
    wts = np.concatenate([np.asarray(w.s).reshape(w.nsteps, -1),
                          np.asarray(w.gamma).reshape(w.nsteps, -1)], axis=1)
    nz = wts[:, :128] != 0.0
    return [sum(1 << m for m in np.nonzero(row)[0]) for row in nz]


def deep_features(keys, masks, nbits):
    """Network input of (key, channel mask) pairs: +1 / -1 for key bits b < nbits, then 1 / 0 per
    channel, 0 past 128."""
    keys = np.asarray(keys, dtype=np.uint64)
    nb = min(nbits, DEEP_IN)
    x = np.zeros((len(keys), DEEP_IN), dtype=np.int64)
    b = np.arange(nb, dtype=np.uint64)
    bits = ((keys[:, None] >> b[None, :]) & np.uint64(1)).astype(np.int64)
    x[:, :nb] = 2 * bits - 1
    nch = DEEP_IN - nb
    ids, table = {}, []
    idx = np.empty(len(masks), dtype=np.int64)
    for i, m in enumerate(masks):
        j = ids.get(m)
        if j is None:
            j = ids[m] = len(table)
            table.append([(m >> c) & 1 for c in range(nch)])
        idx[i] = j
    if nch > 0 and len(table):
        x[:, nb:] = np.asarray(table, dtype=np.int64)[idx]
    return x


def log_plain_run(ctx, w, capacity):
    """Run workload `w` on `ctx` from its current state to the end with the plain comb on the
    streamed path, logging its spawn events; returns (events, total drawn)."""
    ctx.log_spawns(capacity)
    s0 = ctx.counters()["step"]
    ctx.run_workload(w, s0, w.nsteps)
    ev, total = ctx.log_read()
    ctx.log_spawns(0)
    return ev, total


def deep_training_set(events, w):
    """Training pairs from spawn events: per (parent key, channel mask of its step), the walkers
    spawned into each column group (|re| + |im| summed over the events), as fractions of that
    pair's total, with the total as the pair's weight."""
    kmask = np.uint64((1 << (2 * w.n)) - 1)
    masks = active_masks(w)
    mid_of_step = {}
    uniq = []
    for s, m in enumerate(masks):
        if m not in mid_of_step:
            mid_of_step[m] = len(uniq)
            uniq.append(m)
    step_mid = np.array([mid_of_step[m] for m in masks], dtype=np.int64)
    keep = (events["group"] >= 1) & (events["group"] <= DEEP_OUT)
    ev = events[keep]
    key = ev["key"] & kmask
    mid = step_mid[ev["step"].astype(np.int64)]
    walkers = np.abs(ev["re"].astype(np.int64)) + np.abs(ev["im"].astype(np.int64))
    pair = key.astype(np.uint64) * np.uint64(len(uniq) + 1) + mid.astype(np.uint64)
    up, inv = np.unique(pair, return_inverse=True)
    Y = np.zeros((len(up), DEEP_OUT))
    np.add.at(Y, (inv, ev["group"].astype(np.int64) - 1), walkers)
    tot = Y.sum(axis=1)
    Y /= tot[:, None]
    pkeys = up // np.uint64(len(uniq) + 1)
    pmids = (up % np.uint64(len(uniq) + 1)).astype(np.int64)
    pmasks = [uniq[i] for i in pmids.tolist()]
    return pkeys, pmasks, Y, tot


def fit_deep(X, Y, wt, G, iters=2500, lr=2e-3, batch=2048, seed=0):
    """Float network (DEEP_IN -> DEEP_HIDDEN relu -> DEEP_HIDDEN relu -> DEEP_OUT) whose weights
    W_g = relu(score_g) give the proposal's group probabilities as the kernel forms them,
    q_g = 1 / (16 (G - 1)) + (15 / 16) W_g / sum W (the floor of every channel, then the rest in
    proportion), fitted to the spawn fractions t_g by the importance-sampling variance
    sum_g t_g^2 / q_g (minimal at q = t), weighted by the pair's walkers wt; Adam.  G: the column
    groups (diagonal included) of each pair's step table."""
    rng = np.random.default_rng(seed)
    X = X.astype(np.float32)
    Y = Y.astype(np.float32)
    wt = (wt / wt.mean()).astype(np.float32)
    ng = np.maximum(np.asarray(G, dtype=np.int64) - 1, 1)
    valid = (np.arange(DEEP_OUT)[None, :] < ng[:, None]).astype(np.float32)
    floor = (1.0 / (16.0 * ng)).astype(np.float32)
    sh = [(DEEP_HIDDEN, DEEP_IN), (DEEP_HIDDEN,), (DEEP_HIDDEN, DEEP_HIDDEN), (DEEP_HIDDEN,),
          (DEEP_OUT, DEEP_HIDDEN), (DEEP_OUT,)]
    params = [rng.normal(0, np.sqrt(2.0 / s[1]), s).astype(np.float32) if len(s) == 2 else
              np.zeros(s, np.float32) for s in sh]
    params[5][:] = 1.0
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    for it in range(1, iters + 1):
        idx = rng.integers(0, len(X), size=min(batch, len(X)))
        x, t, ww, vd, fl = X[idx], Y[idx], wt[idx][:, None], valid[idx], floor[idx][:, None]
        W1, b1, W2, b2, W3, b3 = params
        a1 = x @ W1.T + b1
        h1 = np.maximum(a1, 0)
        a2 = h1 @ W2.T + b2
        h2 = np.maximum(a2, 0)
        out = h2 @ W3.T + b3
        Wg = (np.maximum(out, 0) + 1e-6) * vd
        Z = Wg.sum(axis=1, keepdims=True)
        q = fl + (15.0 / 16.0) * Wg / Z
        # L = sum_g t^2 / q over the valid groups; dL/dW_k = (15/16) / Z (dq_k - sum_g dq_g W_g / Z)
        dq = -(t * t) / (q * q) * vd
        dW = (15.0 / 16.0) / Z * (dq - (dq * Wg).sum(axis=1, keepdims=True) / Z) * vd
        d = ww * dW * (out > 0) / len(x)
        gW3, gb3 = d.T @ h2, d.sum(0)
        d2 = (d @ W3) * (a2 > 0)
        gW2, gb2 = d2.T @ h1, d2.sum(0)
        d1 = (d2 @ W2) * (a1 > 0)
        gW1, gb1 = d1.T @ x, d1.sum(0)
        for i, gr in enumerate([gW1, gb1, gW2, gb2, gW3, gb3]):
            m[i] = 0.9 * m[i] + 0.1 * gr
            v[i] = 0.999 * v[i] + 0.001 * gr * gr
            params[i] -= lr * (m[i] / (1 - 0.9 ** it)) / (np.sqrt(v[i] / (1 - 0.999 ** it)) + 1e-8)
    return params


def proposal_variance(W, Y, G):
    """Mean over pairs of sum_g t_g^2 / q_g for integer weights W (>= 0) under the kernel's
    thresholds (all-zero weights count as all one): 1 at q = t, larger otherwise."""
    ng = np.maximum(np.asarray(G, dtype=np.int64) - 1, 1)
    valid = np.arange(DEEP_OUT)[None, :] < ng[:, None]
    Wv = np.where(valid, np.maximum(W, 0).astype(np.float64), 0.0)
    Z = Wv.sum(axis=1, keepdims=True)
    Wv = np.where(Z > 0, Wv, valid.astype(np.float64))
    Z = Wv.sum(axis=1, keepdims=True)
    q = 1.0 / (16.0 * ng[:, None]) + (15.0 / 16.0) * Wv / Z
    return float(np.mean(np.where(valid, Y * Y / q, 0.0).sum(axis=1)))


def _shift_for(a):
    """Right shift that brings the 99.9th percentile of the positive activations near 127."""
    pos = a[a > 0]
    if len(pos) == 0:
        return 0
    top = float(np.percentile(pos, 99.9))
    return int(max(0, np.ceil(np.log2(max(top, 1.0) / 127.0))))


def quantize_deep(params, X):
    """Integer network of the ABI from the float one: each layer's weights in units of its
    max|w| / 127, hidden shifts from the activations of the training inputs, biases in the
    matching units."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    u1 = max(np.abs(W1).max(), 1e-12) / 127.0
    w1q = np.clip(np.rint(W1 / u1), -127, 127).astype(np.int8)
    b1q = np.clip(np.rint(b1 / u1), -(1 << 30), 1 << 30).astype(np.int64)
    a1 = X @ w1q.T.astype(np.int64) + b1q
    s1 = _shift_for(a1)
    h1 = np.minimum(np.where(a1 > 0, a1, 0) >> s1, 127)
    unit1 = u1 * (1 << s1)                 # float value of one unit of h1
    u2 = max(np.abs(W2).max(), 1e-12) / 127.0
    w2q = np.clip(np.rint(W2 / u2), -127, 127).astype(np.int8)
    b2q = np.clip(np.rint(b2 / (u2 * unit1)), -(1 << 30), 1 << 30).astype(np.int64)
    a2 = h1 @ w2q.T.astype(np.int64) + b2q
    s2 = _shift_for(a2)
    unit2 = u2 * unit1 * (1 << s2)
    u3 = max(np.abs(W3).max(), 1e-12) / 127.0
    w3q = np.clip(np.rint(W3 / u3), -127, 127).astype(np.int8)
    b3q = np.clip(np.rint(b3 / (u3 * unit2)), -(1 << 24), 1 << 24).astype(np.int32)
    return (w1q, b1q.astype(np.int32), w2q, b2q.astype(np.int32), w3q, b3q, s1, s2)


def deep_scores(net, X):
    """Integer scores of the quantized deeper network (the ABI's definition), for inspection."""
    w1, b1, w2, b2, w3, b3, s1, s2 = net
    a1 = X @ w1.T.astype(np.int64) + b1
    h1 = np.minimum(np.where(a1 > 0, a1, 0) >> s1, 127)
    a2 = h1 @ w2.T.astype(np.int64) + b2
    h2 = np.minimum(np.where(a2 > 0, a2, 0) >> s2, 127)
    return h2 @ w3.T.astype(np.int64) + b3


def train_deep(ctx, w, capacity=16_000_000, max_pairs=1_500_000, seed=0):
    """Spawn events of a plain run of `w` on `ctx` (from its current state), then the fit and the
    quantization.  Returns (net for QMC.set_proposal_deep, info): events drawn and stored,
    training pairs, and the mean importance-sampling variance factor sum_g t_g^2 / q_g of the
    integer network on the training pairs (1 = the spawn fractions exactly; uniform and the
    fractions themselves given beside it)."""
    ev, total = log_plain_run(ctx, w, capacity)
    keys, masks, Y, tot = deep_training_set(ev, w)
    rng = np.random.default_rng(seed)
    if len(keys) > max_pairs:
        pick = rng.choice(len(keys), size=max_pairs, replace=False)
        keys, masks, Y, tot = keys[pick], [masks[i] for i in pick], Y[pick], tot[pick]
    # column groups of each pair's step table (the library's host table builder)
    groups_of_mask = {}
    for k, m in enumerate(active_masks(w)):
        if m not in groups_of_mask:
            tab = binding.coeff_table(w.n, w.dt, w.h, w.lops, w.s[k], w.gamma[k])
            groups_of_mask[m] = len(tab["gxmask"])
    G = np.array([groups_of_mask[m] for m in masks], dtype=np.int64)
    X = deep_features(keys, masks, 2 * w.n)
    # every pair counts the same: the few parents with up to 1e8 walkers would otherwise decide
    # the fit alone (their groups follow the same rules as everyone's)
    params = fit_deep(X, Y, np.ones(len(keys)), G, lr=1e-3, seed=seed)
    net = quantize_deep(params, X)
    sc = deep_scores(net, X)
    return net, {"events_drawn": int(total), "events_stored": int(len(ev)),
                 "training_pairs": int(len(keys)), "shifts": [int(net[6]), int(net[7])],
                 "variance_factor": proposal_variance(sc, Y, G),
                 "variance_factor_uniform": proposal_variance(np.ones_like(sc), Y, G),
                 "variance_factor_exact": proposal_variance(np.rint(Y * (1 << 20)), Y, G)}
