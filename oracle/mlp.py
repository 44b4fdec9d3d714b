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


def backward(X, H1, H2, dY, P, emulate_bf16=True, given=None, stages=None):
    """Gradients of the loss with respect to every parameter (chain rule
    through the three layers, ReLU derivative = [activation > 0]).

    `given` may hold stored intermediates to use instead of recomputing
    them -- "dY16" (the logit gradient as handed to the products), "dH2",
    "dH1" (hidden-layer gradients as stored) -- so that each layer can be
    checked on its own inputs; `stages`, if a dict, receives the values this
    function computed for those three before rounding ("dH2_raw",
    "dH1_raw") and after ("dY16", "dH2", "dH1")."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    given = given or {}
    st = {} if stages is None else stages
    st["dY16"] = r(dY)
    dYr = given.get("dY16", st["dY16"])
    g = {"W3": H2.T @ dYr, "b3": dY.sum(axis=0)}
    st["dH2_raw"] = (dYr @ r(P["W3"]).T) * (H2 > 0)
    st["dH2"] = r(st["dH2_raw"])
    dH2 = given.get("dH2", st["dH2"])
    g["W2"] = H1.T @ dH2
    g["b2"] = st["dH2_raw"].sum(axis=0)
    st["dH1_raw"] = (dH2 @ r(P["W2"]).T) * (H1 > 0)
    st["dH1"] = r(st["dH1_raw"])
    dH1 = given.get("dH1", st["dH1"])
    g["W1"] = r(X).T @ dH1
    g["b1"] = st["dH1_raw"].sum(axis=0)
    return g


def adam(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def head_softmax(Y):
    """Per-head softmax probabilities of (n, 64) logits."""
    Y = np.asarray(Y, dtype=np.float64)
    p = np.zeros_like(Y)
    for h in range(6):
        a, e = STARTS[h], STARTS[h + 1]
        z = np.exp(Y[:, a:e] - Y[:, a:e].max(axis=1, keepdims=True))
        p[:, a:e] = z / z.sum(axis=1, keepdims=True)
    return p


def score(Y, rarity):
    """Novelty score: expected rarity of the predicted class, summed over
    the six heads, s = sum_h sum_{j in h} p_j rarity_j."""
    p = head_softmax(Y)
    rarity = np.asarray(rarity, dtype=np.float64)
    return sum(p[:, STARTS[h]:STARTS[h + 1]] @ rarity[STARTS[h]:STARTS[h + 1]] for h in range(6))


def score_grad(Y, rarity):
    """d score / d Y: within head h, d/dY_j of sum_i p_i r_i is
    p_j (r_j - s_h) with s_h = sum_i p_i r_i (derivative of the softmax,
    dp_i/dY_j = p_i ([i = j] - p_j))."""
    p = head_softmax(Y)
    rarity = np.asarray(rarity, dtype=np.float64)
    g = np.zeros_like(p)
    for h in range(6):
        a, e = STARTS[h], STARTS[h + 1]
        sh = p[:, a:e] @ rarity[a:e]
        g[:, a:e] = p[:, a:e] * (rarity[a:e][None, :] - sh[:, None])
    return g


def input_gradient(Y, H1, H2, P, rarity, emulate_bf16=True, given=None, stages=None):
    """d score(forward(X)) / d X for the forward pass that produced (Y, H1,
    H2): the logit gradient of the score (stored in bfloat16 when
    emulating), through W3 and the second ReLU, through W2 and the first
    ReLU, then through W1 (the result is not rounded).  `given` / `stages`
    as in backward, with keys "dY16", "dH2", "dH1" (and "dH2_raw",
    "dH1_raw" before rounding)."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    given = given or {}
    st = {} if stages is None else stages
    st["dY16"] = r(score_grad(Y, rarity))
    dY = given.get("dY16", st["dY16"])
    st["dH2_raw"] = (dY @ r(P["W3"]).T) * (H2 > 0)
    st["dH2"] = r(st["dH2_raw"])
    dH2 = given.get("dH2", st["dH2"])
    st["dH1_raw"] = (dH2 @ r(P["W2"]).T) * (H1 > 0)
    st["dH1"] = r(st["dH1_raw"])
    dH1 = given.get("dH1", st["dH1"])
    return dH1 @ r(P["W1"]).T


# ------------------------------------------------------- proposal sampling
# The mutation kernels draw their random bits from a counter-based
# generator: the SplitMix64 output function (Steele, Lea, Flood 2014,
# "Fast splittable pseudorandom number generators") applied to a key, with
# key(seed, k, f) = mix(seed XOR mix(k * 0x100000001B3 + f)) for flip f of
# candidate k.  Written here from that definition (Python integers mod 2^64).

_M64 = (1 << 64) - 1


def splitmix_mix(z):
    """SplitMix64 output for state increment z: add the golden gamma, then
    the two xor-shift-multiply rounds and a final xor-shift."""
    z = (z + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def flip_key(seed, k, f):
    return splitmix_mix((seed ^ splitmix_mix((k * 0x100000001B3 + f) & _M64)) & _M64)


def _toggle(lo, hi, b):
    return (lo ^ (1 << b), hi) if b < 64 else (lo, hi ^ (1 << (b - 64)))


def mutate(parents, n, n_bits, flips, seed):
    """Uniform mutants: candidate k copies parent k mod len(parents) and
    toggles `flips` bits, flip f toggling bit 1 + key mod (n_bits - 1)
    (bit 0 is never touched).  Returns (n, 2) uint64."""
    par = np.asarray(parents, dtype=np.uint64).reshape(-1, 2)
    out = np.zeros((n, 2), dtype=np.uint64)
    for k in range(n):
        lo, hi = int(par[k % len(par), 0]), int(par[k % len(par), 1])
        for f in range(flips):
            lo, hi = _toggle(lo, hi, 1 + flip_key(seed, k, f) % (n_bits - 1))
        out[k] = (lo, hi)
    return out


def flip_cdf(parents, dX, n_bits, temp, explore):
    """Flip distribution of each parent from the input gradient dX of the
    novelty score: the first-order change of the score when bit j flips is
    gain_j = -2 x_j dX_j (x_j = +1 for '+', -1 for '-'); bit j in
    [1, n_bits) gets probability (1 - explore) softmax_j(gain / (temp
    max_j |gain_j|)) + explore / (n_bits - 1).  Returns the (n, 64)
    cumulative table: entry j = P(bit <= j), entry 0 = 0, entries from
    n_bits - 1 on = 1."""
    par = np.asarray(parents, dtype=np.uint64).reshape(-1, 2)
    dX = np.asarray(dX, dtype=np.float64)
    out = np.zeros((len(par), 64))
    for p in range(len(par)):
        x = np.array([1.0 if not ((int(par[p, j // 64]) >> (j % 64)) & 1) else -1.0 for j in range(n_bits)])
        gain = -2.0 * x[1:] * dX[p, 1:n_bits]
        scale = temp * np.abs(gain).max()
        # all gains zero: the softmax of equal values is uniform
        w = np.exp((gain - gain.max()) / scale) if scale > 0 else np.ones_like(gain)
        prob = (1.0 - explore) * w / w.sum() + explore / (n_bits - 1)
        out[p, 1:n_bits - 1] = np.cumsum(prob)[:n_bits - 2]
        out[p, n_bits - 1:] = 1.0
    return out


def mutate_cdf(parents, cdf, n, flips, seed):
    """Guided mutants: candidate k copies parent p = k mod len(parents) and
    toggles `flips` bits, flip f drawing u = (key >> 40) / 2^24 and toggling
    the bit b = min{j >= 1 : u < cdf[p][j]} (inverse transform sampling;
    bit 63 if there is none).  The comparison is made in binary32, the
    precision the table is stored in."""
    par = np.asarray(parents, dtype=np.uint64).reshape(-1, 2)
    c = np.asarray(cdf, dtype=np.float32)
    out = np.zeros((n, 2), dtype=np.uint64)
    for k in range(n):
        p = k % len(par)
        lo, hi = int(par[p, 0]), int(par[p, 1])
        for f in range(flips):
            u = np.float32((flip_key(seed, k, f) >> 40) / 16777216.0)   # exact in binary32
            above = [j for j in range(1, 64) if u < c[p, j]]
            lo, hi = _toggle(lo, hi, above[0] if above else 63)
        out[k] = (lo, hi)
    return out


def bin_floats(x, lo, hi, bins):
    """Counts of x in the bins [lo + b w, lo + (b+1) w), w = (hi - lo) /
    bins, values outside clamped into the end bins; the bin index is
    floor((x - lo) / (hi - lo) * bins) evaluated in binary32, the
    precision of the scores (each operation rounded to nearest)."""
    x = np.asarray(x, dtype=np.float32)
    lo32, hi32 = np.float32(lo), np.float32(hi)
    t = ((x - lo32) / (hi32 - lo32)) * np.float32(bins)
    b = np.clip(np.floor(t).astype(np.int64), 0, bins - 1)
    return np.bincount(b, minlength=bins)


def select(score_, cand, threshold):
    """The candidates whose score exceeds the threshold (as a set of rows,
    in input order) and their number."""
    keep = np.asarray(score_, dtype=np.float32) > np.float32(threshold)
    return np.asarray(cand, dtype=np.uint64).reshape(-1, 2)[keep], int(keep.sum())
