"""FP64 oracle of the learned pre-screen -- TEST INFRASTRUCTURE ONLY.

A message-passing network over the ligand graph followed by an MLP predicts
a ligand's docking score from its topology, so that full docking (the
paper's screening workload, Sec. 1 and Sec. 2.2: many ligands against one
receptor) runs only on the ligands it ranks best.  The paper has no such
network; its form (3 message-passing layers of width 128, sum pooling, a
128-256-256-1 MLP, BF16 operands with FP32 accumulation, MSE plus a
pairwise ranking loss, Adam) is the target configuration's.

Everything is float64.  With ``bf16=True`` values are rounded to bfloat16
(round to nearest even) at exactly the points where the GPU path stores
BF16 tensors, so the two can be compared; with ``bf16=False`` the network is
a smooth function and its gradient is checked by finite differences.

Definitions (shared reading, implemented independently on the GPU):
  features x (32 per atom): one-hot type [0,16), q, |q|, one-hot degree
    0,1,2,3,>=4 at [18,23), (rotatable bonds at the atom)/2 at 23, 1 at 31
  H0 = r(relu(X W0 + b0));  for l=1..3: M_l = r(A H_{l-1}),
    H_l = r(relu([H_{l-1} | M_l] W_l + b_l))   (A: bond adjacency)
  g = r(sum_atoms H3); z1 = r(relu(g U1 + c1)); z2 = r(relu(z1 U2 + c2))
  p = z2 U3 + c3                                       (r = BF16 rounding)
  loss over a minibatch with standardised labels y:
    mean (p - y)^2 + lam * mean_{y_i < y_j} softplus((p_i - p_j) / tau)
"""
from __future__ import annotations

import numpy as np

F_IN, WIDTH, HID = 32, 128, 256
N_LAYERS = 3
LAM, TAU = 1.0, 0.5
ADAM = dict(lr=1e-3, b1=0.9, b2=0.999, eps=1e-8)

# parameter tensors in their flattened order: (name, shape)
PARAM_SHAPES = ([("W0", (F_IN, WIDTH)), ("b0", (WIDTH,))] +
                [(n, s) for l in range(1, N_LAYERS + 1)
                 for n, s in ((f"W{l}", (2 * WIDTH, WIDTH)), (f"b{l}", (WIDTH,)))] +
                [("U1", (WIDTH, HID)), ("c1", (HID,)), ("U2", (HID, HID)), ("c2", (HID,)),
                 ("U3", (HID, 1)), ("c3", (1,))])
N_PARAMS = int(sum(np.prod(s) for _, s in PARAM_SHAPES))


def bf16(x):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(theta):
    out, o = {}, 0
    for n, s in PARAM_SHAPES:
        k = int(np.prod(s))
        out[n] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(s)
        o += k
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[n], dtype=np.float64).reshape(-1) for n, _ in PARAM_SHAPES])


def features(lig):
    """Atom features and adjacency lists of one ligand (input atom order)."""
    n = lig.n_atoms
    X = np.zeros((n, F_IN))
    deg = np.zeros(n, dtype=int)
    rot = np.zeros(n)
    nbr = [[] for _ in range(n)]
    for (a, b), r in zip(lig.bonds, lig.rotatable):
        a, b = int(a), int(b)
        nbr[a].append(b)
        nbr[b].append(a)
        deg[a] += 1
        deg[b] += 1
        if r:
            rot[a] += 1
            rot[b] += 1
    for i in range(n):
        X[i, int(lig.types[i])] = 1.0
        q = float(lig.charges[i])
        X[i, 16] = q
        X[i, 17] = abs(q)
        X[i, 18 + min(deg[i], 4)] = 1.0
        X[i, 23] = rot[i] / 2.0
        X[i, 31] = 1.0
    return X, nbr


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def _adj(nbr, H):
    return np.stack([H[nb].sum(axis=0) if nb else np.zeros(H.shape[1]) for nb in nbr])


def forward(theta, graphs, bf16_on=True, keep=False):
    """graphs: list of (X, nbr).  Returns predictions p [B] (and the saved
    activations when keep=True)."""
    P = unflatten(theta)
    W = {k: _r(v, bf16_on) for k, v in P.items() if k[0] in "WU"}
    cache = []
    G = []
    for X, nbr in graphs:
        Xr = _r(X, bf16_on)
        H = _r(np.maximum(Xr @ W["W0"] + P["b0"], 0.0), bf16_on)
        Hs, Ms = [H], [None]
        for l in range(1, N_LAYERS + 1):
            M = _r(_adj(nbr, H), bf16_on)
            H = _r(np.maximum(np.concatenate([H, M], axis=1) @ W[f"W{l}"] + P[f"b{l}"], 0.0), bf16_on)
            Hs.append(H)
            Ms.append(M)
        G.append(_r(H.sum(axis=0), bf16_on))
        cache.append((Xr, nbr, Hs, Ms))
    g = np.stack(G)
    z1 = _r(np.maximum(g @ W["U1"] + P["c1"], 0.0), bf16_on)
    z2 = _r(np.maximum(z1 @ W["U2"] + P["c2"], 0.0), bf16_on)
    p = (z2 @ W["U3"])[:, 0] + P["c3"][0]
    if keep:
        return p, dict(cache=cache, g=g, z1=z1, z2=z2, W=W)
    return p


def loss_and_dp(p, y, lam=LAM, tau=TAU):
    """MSE + lam * mean over pairs (y_i < y_j) of softplus((p_i - p_j)/tau)."""
    p = np.asarray(p, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    B = len(p)
    d = p - y
    loss = np.mean(d * d)
    dp = 2.0 * d / B
    better = y[:, None] < y[None, :]            # (i, j): i should score lower than j
    npairs = int(better.sum())
    if npairs and lam:
        z = (p[:, None] - p[None, :]) / tau
        sp = np.logaddexp(0.0, z)
        loss += lam * sp[better].sum() / npairs
        s = 1.0 / (1.0 + np.exp(-z))
        w = np.where(better, s, 0.0) / tau * lam / npairs
        dp += w.sum(axis=1) - w.sum(axis=0)
    return loss, dp


def backward(theta, graphs, dp, bf16_on=True):
    """Gradient of sum_i dp_i * p_i with respect to the flattened parameters."""
    p, c = forward(theta, graphs, bf16_on, keep=True)
    W, g, z1, z2 = c["W"], c["g"], c["z1"], c["z2"]
    dp = np.asarray(dp, dtype=np.float64)
    gr = {n: np.zeros(s) for n, s in PARAM_SHAPES}
    gr["U3"] = (z2.T @ dp)[:, None]
    gr["c3"] = np.array([dp.sum()])
    dz2 = _r(np.outer(dp, W["U3"][:, 0]) * (z2 > 0), bf16_on)
    gr["U2"] = z1.T @ dz2
    gr["c2"] = dz2.sum(axis=0)
    dz1 = _r((dz2 @ W["U2"].T) * (z1 > 0), bf16_on)
    gr["U1"] = g.T @ dz1
    gr["c1"] = dz1.sum(axis=0)
    dg = _r(dz1 @ W["U1"].T, bf16_on)
    for b, (Xr, nbr, Hs, Ms) in enumerate(c["cache"]):
        n = Xr.shape[0]
        dH = np.tile(dg[b], (n, 1))
        for l in range(N_LAYERS, 0, -1):
            dP = _r(dH, bf16_on) * (Hs[l] > 0)
            HM = np.concatenate([Hs[l - 1], Ms[l]], axis=1)
            gr[f"W{l}"] += HM.T @ dP
            gr[f"b{l}"] += dP.sum(axis=0)
            dHM = _r(dP @ W[f"W{l}"].T, bf16_on)
            dH = dHM[:, :WIDTH] + _adj(nbr, dHM[:, WIDTH:])
        dP0 = _r(dH, bf16_on) * (Hs[0] > 0)
        gr["W0"] += Xr.T @ dP0
        gr["b0"] += dP0.sum(axis=0)
    return flatten(gr), p


def adam_step(theta, grad, m, v, t, lr=ADAM["lr"], b1=ADAM["b1"], b2=ADAM["b2"], eps=ADAM["eps"]):
    """One Adam update (step t >= 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    d = {}
    for n, s in PARAM_SHAPES:
        if n[0] in "WU":
            lim = np.sqrt(6.0 / s[0])
            d[n] = rng.uniform(-lim, lim, size=s)
        else:
            d[n] = np.zeros(s)
    return flatten(d)


# ---------------------------------------------------------------------------
# FP32 emulation: the flip noise of the rounding points above.
#
# The GPU path rounds to BF16 where the oracle does but accumulates in FP32,
# in an order of its own.  Every sum whose exact value lies within the FP32
# accumulation error of a BF16 rounding midpoint can round the other way, and
# such one-ulp differences travel on through the network; every graph has
# thousands of such sums, so no result is free of them.  `emulate_fp32` is a
# second, independent implementation of the same definition in float32: the
# products of BF16 values are exact in float32 and every sum runs in float32
# in a randomly permuted order (a different order per seed), the pooled sum
# in float64 (exact), the loss and its derivative in float32.  The spread of
# its results over seeds around the FP64 oracle is the size of the flip noise
# that any FP32-accumulating implementation of these rounding points shows;
# the GPU tests derive their tolerances from it before measuring.
# ---------------------------------------------------------------------------
def _perm_mm(A, B, rng):
    """float32 A @ B with the summed dimension in a random order."""
    k = A.shape[1]
    o = rng.permutation(k)
    return np.asarray(A, np.float32)[:, o] @ np.asarray(B, np.float32)[o, :]


def _perm_sum(A, rng, axis=0):
    """float32 sequential sum along `axis` in a random order."""
    A = np.asarray(A, np.float32)
    o = rng.permutation(A.shape[axis])
    return np.cumsum(np.take(A, o, axis=axis), axis=axis, dtype=np.float32).take(-1, axis=axis) \
        if A.shape[axis] else np.zeros(np.delete(A.shape, axis), np.float32)


def _adj32(nbr, H, rng, extra=None):
    out = np.zeros((len(nbr), H.shape[1]), np.float32)
    for i, nb in enumerate(nbr):
        rows = [H[j] for j in nb] + ([extra[i]] if extra is not None else [])
        if rows:
            out[i] = _perm_sum(np.stack(rows), rng)
    return out


def emulate_fp32(theta, graphs, ys=None, seed=0, lam=LAM, tau=TAU, bf16_on=True):
    """Predictions (and with labels ys: loss, flattened gradient) of the
    network with BF16 rounding at the oracle's points (bf16_on) and float32
    sums in a random order fixed by `seed`."""
    rng = np.random.default_rng(seed)
    P = unflatten(theta)
    f32 = lambda a: np.asarray(a, np.float32)
    r = (lambda a: f32(bf16(a))) if bf16_on else f32
    W = {k: r(v) for k, v in P.items() if k[0] in "WU"}
    b32 = {k: f32(v) for k, v in P.items() if k[0] in "bc"}
    cache, G = [], []
    for X, nbr in graphs:
        Xr = r(X)
        H = r(np.maximum(_perm_mm(Xr, W["W0"], rng) + b32["b0"], 0.0))
        Hs, Ms = [H], [None]
        for l in range(1, N_LAYERS + 1):
            M = r(_adj32(nbr, H, rng))
            H = r(np.maximum(_perm_mm(np.concatenate([H, M], axis=1), W[f"W{l}"], rng) + b32[f"b{l}"], 0.0))
            Hs.append(H)
            Ms.append(M)
        G.append(r(H.astype(np.float64).sum(axis=0)))
        cache.append((Xr, nbr, Hs, Ms))
    g = np.stack(G)
    z1 = r(np.maximum(_perm_mm(g, W["U1"], rng) + b32["c1"], 0.0))
    z2 = r(np.maximum(_perm_mm(z1, W["U2"], rng) + b32["c2"], 0.0))
    p = _perm_mm(z2, W["U3"], rng)[:, 0] + b32["c3"][0]
    if ys is None:
        return p.astype(np.float64)
    y = f32(ys)
    B = len(y)
    d = p - y
    better = y[:, None] < y[None, :]
    npairs = np.float32(better.sum())
    wr = np.float32(lam) / npairs if npairs else np.float32(0.0)
    z = (p[:, None] - p[None, :]) / np.float32(tau)
    li = d * d / np.float32(B) + wr * np.where(better, np.maximum(z, 0) + np.log1p(np.exp(-np.abs(z))), 0).sum(1)
    with np.errstate(over="ignore"):
        sgm = np.float32(1.0) / (np.float32(1.0) + np.exp(-z))
    gi = np.float32(2.0) * d / np.float32(B) + (wr / np.float32(tau)) * (np.where(better, sgm, 0).sum(1)
                                                                          - np.where(better.T, sgm.T, 0).sum(1))
    loss = _perm_sum(li, rng)
    dp = f32(gi)
    gr = {}
    U3 = W["U3"][:, 0]
    gr["U3"] = _perm_mm(z2.T, dp[:, None], rng)
    gr["c3"] = np.array([_perm_sum(dp, rng)])
    dz2 = r(dp[:, None] * U3[None, :]) * (z2 > 0)
    ones = np.ones((1, B), np.float32)
    gr["U2"] = _perm_mm(z1.T, dz2, rng)
    gr["c2"] = _perm_mm(ones, dz2, rng)[0]
    dz1 = r(_perm_mm(dz2, W["U2"].T, rng) * (z1 > 0))
    gr["U1"] = _perm_mm(g.T, dz1, rng)
    gr["c1"] = _perm_mm(ones, dz1, rng)[0]
    dg = r(_perm_mm(dz1, W["U1"].T, rng))
    parts = {n: [] for n, _ in PARAM_SHAPES if n[0] in "Wb"}
    for b, (Xr, nbr, Hs, Ms) in enumerate(cache):
        n = Xr.shape[0]
        dH = np.tile(dg[b], (n, 1))
        on = np.ones((1, n), np.float32)
        for l in range(N_LAYERS, 0, -1):
            dP = r(dH) * (Hs[l] > 0)
            HM = np.concatenate([Hs[l - 1], Ms[l]], axis=1)
            parts[f"W{l}"].append(_perm_mm(HM.T, dP, rng))
            parts[f"b{l}"].append(_perm_mm(on, dP, rng)[0])
            dHM = r(_perm_mm(dP, W[f"W{l}"].T, rng))
            dH = _adj32(nbr, dHM[:, WIDTH:], rng, extra=dHM[:, :WIDTH])
        dP0 = r(dH) * (Hs[0] > 0)
        parts["W0"].append(_perm_mm(Xr.T, dP0, rng))
        parts["b0"].append(_perm_mm(on, dP0, rng)[0])
    for k, v in parts.items():
        gr[k] = _perm_sum(np.stack(v), rng)
    return p.astype(np.float64), float(loss), flatten(gr)
