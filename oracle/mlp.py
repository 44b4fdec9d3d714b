"""CPU oracle of the learned proposal's network -- TEST INFRASTRUCTURE ONLY.

Plain numpy float64 reference of the small MLP that ranks candidate sign
distributions (inputs: the +-1 signs of a mask; outputs: 64 logits in six
softmax heads predicting features of the scheme; Sec. 3 explains why sweeps
over sign distributions dominate the search).  Only the tests may import
this module; the product's kernels never do.

Where the GPU path stores a value in bfloat16 (weights, the +-1 inputs, the
hidden activations handed to the next product, the output gradient) this
reference rounds it the same way, so the remaining GPU/CPU difference is the
FP32 accumulation order.  bfloat16 rounding: the upper 16 bits of an IEEE-754
binary32 value, rounded to nearest with ties to even.

Heads (64 logits): number of ovals clamped to 22 (23 classes), deepest
nesting level clamped to 4 (5 classes), and for depths 1..4 the number of
ovals at that depth in buckets 0,1,2,3,4,5-6,7-9,10-14,15+ (9 classes each).
"""
from __future__ import annotations

import numpy as np

HEADS = (23, 5, 9, 9, 9, 9)
STARTS = np.concatenate([[0], np.cumsum(HEADS)])
WIDTH_IN = 64   # 45 signs at d = 8, zero-padded
HIDDEN = 512
OUT = 64


def bf16(x):
    """Round float64/float32 values to bfloat16 (returned as float64)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return ((r << 16).astype(np.uint32)).view(np.float32).astype(np.float64)


def encode(masks2, n_bits, width=WIDTH_IN):
    """+1 for a '+' sign (bit 0), -1 for '-', 0 in the padding columns."""
    m = np.asarray(masks2, dtype=np.uint64).reshape(-1, 2)
    X = np.zeros((len(m), width))
    for j in range(n_bits):
        word = m[:, j // 64]
        bit = (word >> np.uint64(j % 64)) & np.uint64(1)
        X[:, j] = np.where(bit == 1, -1.0, 1.0)
    return X


def bucket9(c):
    if c <= 4:
        return c
    if c <= 6:
        return 5
    if c <= 9:
        return 6
    if c <= 14:
        return 7
    return 8


def features(codes2):
    """Targets of the six heads from (n,2) uint64 scheme codes."""
    out = np.zeros((len(codes2), 6), dtype=np.int64)
    for k, (lo, hi) in enumerate(np.asarray(codes2, dtype=np.uint64)):
        c = (int(lo) | (int(hi) << 64)) & ((1 << 127) - 1)
        w = bin(c)[3:]
        depth = maxd = ovals = 0
        cnt = [0, 0, 0, 0]
        for ch in w:
            if ch == "1":
                depth += 1
                ovals += 1
                maxd = max(maxd, depth)
                if depth <= 4:
                    cnt[depth - 1] += 1
            else:
                depth -= 1
        out[k] = [min(ovals, 22), min(maxd, 4)] + [bucket9(x) for x in cnt]
    return out


def init_params(seed=0, n_in=45):
    """He-uniform initial weights (fp32 masters), zero biases."""
    rng = np.random.default_rng(seed)

    def he(fan_in, shape):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=shape).astype(np.float32).astype(np.float64)

    W1 = he(n_in, (WIDTH_IN, HIDDEN))
    W1[n_in:] = 0.0
    return {"W1": W1, "b1": np.zeros(HIDDEN), "W2": he(HIDDEN, (HIDDEN, HIDDEN)), "b2": np.zeros(HIDDEN),
            "W3": he(HIDDEN, (HIDDEN, OUT)), "b3": np.zeros(OUT)}


def forward(X, P, emulate_bf16=True):
    """Returns (Y, H1, H2) with H1, H2 as handed to the next product."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    H1 = r(np.maximum(r(X) @ r(P["W1"]) + P["b1"], 0.0))
    H2 = r(np.maximum(H1 @ r(P["W2"]) + P["b2"], 0.0))
    Y = H2 @ r(P["W3"]) + P["b3"]
    return Y, H1, H2


def softmax_xent(Y, labels):
    """Mean over the batch of the summed per-head cross-entropies, and its
    gradient with respect to the logits."""
    n = len(Y)
    loss = 0.0
    dY = np.zeros_like(Y)
    for h in range(6):
        s, e = STARTS[h], STARTS[h + 1]
        z = Y[:, s:e] - Y[:, s:e].max(axis=1, keepdims=True)
        p = np.exp(z)
        p /= p.sum(axis=1, keepdims=True)
        t = labels[:, h]
        loss += -np.log(p[np.arange(n), t]).sum()
        g = p.copy()
        g[np.arange(n), t] -= 1.0
        dY[:, s:e] = g
    return loss / n, dY / n


def backward(X, H1, H2, dY, P, emulate_bf16=True):
    """Gradients of the loss with respect to every parameter."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    dYr = r(dY)
    g = {"W3": H2.T @ dYr, "b3": dY.sum(axis=0)}
    dH2 = r((dYr @ r(P["W3"]).T) * (H2 > 0))
    g["W2"] = H1.T @ dH2
    g["b2"] = ((dYr @ r(P["W3"]).T) * (H2 > 0)).sum(axis=0)
    dH1 = r((dH2 @ r(P["W2"]).T) * (H1 > 0))
    g["W1"] = r(X).T @ dH1
    g["b1"] = ((dH2 @ r(P["W2"]).T) * (H1 > 0)).sum(axis=0)
    return g


def adam(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def score(Y, rarity):
    """Expected rarity of the predicted classes, summed over heads."""
    s = np.zeros(len(Y))
    for h in range(6):
        a, e = STARTS[h], STARTS[h + 1]
        z = Y[:, a:e] - Y[:, a:e].max(axis=1, keepdims=True)
        p = np.exp(z)
        p /= p.sum(axis=1, keepdims=True)
        s += p @ rarity[a:e]
    return s
