"""Learned sign-distribution proposal (binding + orchestration).

A small MLP (inputs: the +-1 signs of a mask; 45 -> 512 -> 512 -> 64, ReLU)
is trained on masks labelled by the exact scheme kernels with six softmax
heads predicting features of the scheme: number of ovals, deepest nesting,
and ovals per nesting depth.  Proposal rounds mutate the witnesses of the
rarest schemes seen so far, rank the mutants by the network's expected
rarity of their features, and hand the best to the exact kernels, which
judge every proposal.  Uniform sampling and the same mutation search with
random ranking are the baselines.

All arithmetic runs in the library's HIP kernels (BF16 matrix-core products
with FP32 accumulation, softmax cross-entropy, Adam, scoring, mutation,
selection); this module only allocates buffers and sequences calls.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import patchwork as pw

HEADS = (23, 5, 9, 9, 9, 9)
WIDTH_IN, HIDDEN, OUT = 64, 512, 64

_bound = False


def _bind():
    global _bound
    if _bound:
        return pw.lib()
    L = pw.lib()
    vp, i32, i64, u64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
    L.pw_mlp_gemm.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, i32, vp, vp, i64, i32, vp, vp, i64, i32, vp, vp]
    L.pw_mlp_encode.argtypes = [vp, i64, i32, i32, vp, vp]
    L.pw_features.argtypes = [vp, i64, vp, vp]
    L.pw_mlp_softmax_xent.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.pw_mlp_colsum.argtypes = [vp, i64, i32, vp, i32, vp]
    L.pw_fill_f32.argtypes = [vp, i64, f32, vp]
    L.pw_label_counts.argtypes = [vp, i64, vp, vp]
    L.pw_mlp_score_grad.argtypes = [vp, vp, i64, vp, vp]
    L.pw_flip_cdf.argtypes = [vp, vp, i64, i64, i32, f32, f32, vp, vp]
    L.pw_mutate_cdf.argtypes = [vp, vp, i64, i64, i32, u64, vp, vp]
    L.pw_mlp_adam.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp, vp]
    L.pw_mlp_score.argtypes = [vp, vp, i64, vp, vp]
    L.pw_to_bf16.argtypes = [vp, i64, vp, vp]
    L.pw_mutate.argtypes = [vp, i64, i64, i32, i32, u64, vp, vp]
    L.pw_select.argtypes = [vp, vp, i64, f32, vp, i64, vp, vp]
    L.pw_random_masks.argtypes = [u64, u64, i64, i32, vp, vp]
    L.pw_bin_floats.argtypes = [vp, i64, f32, f32, i32, vp, vp]
    L.pw_bf16_transpose.argtypes = [vp, i64, i64, vp, vp]
    for n in ("pw_mlp_gemm", "pw_mlp_encode", "pw_features", "pw_mlp_softmax_xent", "pw_mlp_colsum",
              "pw_mlp_adam", "pw_mlp_score", "pw_to_bf16", "pw_mutate", "pw_select",
              "pw_random_masks", "pw_bin_floats", "pw_fill_f32", "pw_mlp_score_grad", "pw_flip_cdf", "pw_mutate_cdf",
              "pw_label_counts", "pw_bf16_transpose"):
        getattr(L, n).restype = i32
    _bound = True
    return L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def gemm(A, a_m, a_k, B, b_k, b_n, M, N, K, C32=None, C16=None, c_m=None, bias=None, gate=None, g_m=0,
         relu=False, accumulate=False, colsum=None):
    """C = A B with element strides (A[m,k] = A[m*a_m + k*a_k], ...);
    colsum (optional) accumulates the column sums of the result."""
    L = _bind()
    pw.check(L.pw_mlp_gemm(_p(A), a_m, a_k, _p(B), b_k, b_n, M, N, K, _p(bias), _p(gate), g_m, int(relu),
                           _p(C32), _p(C16), N if c_m is None else c_m, int(accumulate), _p(colsum), _s()))


def encode(masks128, n, n_bits, width=WIDTH_IN):
    import torch

    X = torch.empty((n, width), dtype=torch.int16, device=masks128.device)
    pw.check(_bind().pw_mlp_encode(_p(masks128), n, n_bits, width, _p(X), _s()))
    return X


def features(codes):
    import torch

    n = codes.shape[0]
    lab = torch.empty((n, 6), dtype=torch.int32, device=codes.device)
    pw.check(_bind().pw_features(_p(codes), n, _p(lab), _s()))
    return lab


def transpose16(x, out=None):
    """(r, c) bf16 (int16) device matrix -> its (c, r) transpose."""
    import torch

    r, c = x.shape
    if out is None:
        out = torch.empty((c, r), dtype=torch.int16, device=x.device)
    pw.check(_bind().pw_bf16_transpose(_p(x), r, c, _p(out), _s()))
    return out


def to_bf16(t32):
    """fp32 device tensor -> bfloat16 bit patterns (int16 tensor)."""
    import torch

    out = torch.empty(t32.shape, dtype=torch.int16, device=t32.device)
    pw.check(_bind().pw_to_bf16(_p(t32), t32.numel(), _p(out), _s()))
    return out


# parameter layout in one flat fp32 buffer (every offset a multiple of 64
# elements, so every matrix view is 256-byte aligned)
LAYOUT = (("W1", (WIDTH_IN, HIDDEN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (HIDDEN, OUT)), ("b3", (OUT,)))


def _offsets():
    off, o = {}, 0
    for k, shp in LAYOUT:
        n = int(np.prod(shp))
        off[k] = (o, n, shp)
        o += n
    return off, o


class MLP:
    """Device parameters in flat buffers: fp32 masters P, gradients G (plus
    one slot for the loss), Adam moments M, V and the bf16 copy W16, each
    with per-tensor views, and W16T, each weight matrix transposed to
    [out][in] so that both operands of a forward product are contiguous
    along K (the products then stage both in 16-byte chunks).  One training
    step is 15 kernel launches: zero G, three forward products, the loss,
    three weight-gradient products, one bias-gradient column sum (the hidden
    layers' bias gradients are summed in the epilogues of the input-gradient
    products), two input-gradient products, one Adam update over all
    parameters and three transposes."""

    def __init__(self, n_in=45, seed=0, device="cuda"):
        import torch

        self.n_in = n_in
        rng = np.random.default_rng(seed)

        def he(fan_in, shape):
            lim = np.sqrt(6.0 / fan_in)
            return rng.uniform(-lim, lim, size=shape).astype(np.float32)

        W1 = he(n_in, (WIDTH_IN, HIDDEN))
        W1[n_in:] = 0.0
        host = {"W1": W1, "b1": np.zeros(HIDDEN, np.float32), "W2": he(HIDDEN, (HIDDEN, HIDDEN)),
                "b2": np.zeros(HIDDEN, np.float32), "W3": he(HIDDEN, (HIDDEN, OUT)), "b3": np.zeros(OUT, np.float32)}
        self.off, self.n_par = _offsets()
        flat = np.concatenate([host[k].reshape(-1) for k, _ in LAYOUT])
        self.Pf = torch.from_numpy(flat).to(device)
        self.Gf = torch.zeros(self.n_par + 64, dtype=torch.float32, device=device)   # + loss slot
        self.Mf = torch.zeros_like(self.Pf)
        self.Vf = torch.zeros_like(self.Pf)
        self.W16f = torch.empty(self.n_par, dtype=torch.int16, device=device)
        self.P = self._views(self.Pf)
        self.G = self._views(self.Gf)
        self.M = self._views(self.Mf)
        self.V = self._views(self.Vf)
        self.W16 = self._views(self.W16f)
        self.W16T = {k: torch.empty((v.shape[1], v.shape[0]), dtype=torch.int16, device=device)
                     for k, v in self.W16.items() if v.dim() == 2}
        self.loss = self.Gf[self.n_par:self.n_par + 1]
        self.step = 0
        self._buf = {}
        self.sync16()

    def _views(self, flat):
        return {k: flat[o:o + n].view(shp) for k, (o, n, shp) in self.off.items()}

    def _buffers(self, n, dev):
        """Activation and gradient buffers for batches of n rows (reused)."""
        import torch

        b = self._buf.get(n)
        if b is None:
            e = lambda shp, dt: torch.empty(shp, dtype=dt, device=dev)
            b = {"H1": e((n, HIDDEN), torch.int16), "H2": e((n, HIDDEN), torch.int16), "Y": e((n, OUT), torch.float32),
                 "dY32": e((n, OUT), torch.float32), "dY16": e((n, OUT), torch.int16),
                 "dH2_16": e((n, HIDDEN), torch.int16), "dH1_16": e((n, HIDDEN), torch.int16),
                 "dX": e((n, WIDTH_IN), torch.float32)}
            self._buf = {n: b}          # keep one batch size
        return b

    def sync16(self):
        """Refresh the bf16 copy from the fp32 masters."""
        pw.check(_bind().pw_to_bf16(_p(self.Pf), self.n_par, _p(self.W16f), _s()))
        self._sync_t()

    def _sync_t(self):
        for k, t in self.W16T.items():
            transpose16(self.W16[k], t)

    def load(self, host):
        """Set parameters from host float arrays (tests)."""
        import torch

        for k, v in host.items():
            self.P[k].copy_(torch.from_numpy(np.asarray(v, dtype=np.float32)))
        self.sync16()

    def forward(self, X16, keep=False, fresh=True):
        """Logits of a batch (fresh buffers unless fresh=False, which reuses
        this network's training buffers)."""
        import torch

        n = X16.shape[0]
        dev = X16.device
        if fresh:
            H1 = torch.empty((n, HIDDEN), dtype=torch.int16, device=dev)
            H2 = torch.empty((n, HIDDEN), dtype=torch.int16, device=dev)
            Y = torch.empty((n, OUT), dtype=torch.float32, device=dev)
        else:
            b = self._buffers(n, dev)
            H1, H2, Y = b["H1"], b["H2"], b["Y"]
        # B(k, n) = W[k][n] = W^T[n][k]: the transposed copies are contiguous along k
        gemm(X16, WIDTH_IN, 1, self.W16T["W1"], 1, WIDTH_IN, n, HIDDEN, WIDTH_IN, C16=H1, bias=self.P["b1"],
             relu=True)
        gemm(H1, HIDDEN, 1, self.W16T["W2"], 1, HIDDEN, n, HIDDEN, HIDDEN, C16=H2, bias=self.P["b2"], relu=True)
        gemm(H2, HIDDEN, 1, self.W16T["W3"], 1, HIDDEN, n, OUT, HIDDEN, C32=Y, bias=self.P["b3"])
        if keep:
            return Y, H1, H2
        return Y

    def backward(self, X16, H1, H2, Y, labels):
        """Loss and parameter gradients (into G, zeroed first) for one batch;
        returns the loss as a one-element device tensor."""
        L = _bind()
        n = X16.shape[0]
        b = self._buffers(n, X16.device)
        pw.check(L.pw_fill_f32(_p(self.Gf), self.Gf.numel(), 0.0, _s()))
        pw.check(L.pw_mlp_softmax_xent(_p(Y), _p(labels), n, _p(b["dY32"]), _p(b["dY16"]), _p(self.loss), _s()))
        # layer 3
        gemm(H2, 1, HIDDEN, b["dY16"], OUT, 1, HIDDEN, OUT, n, C32=self.G["W3"], accumulate=True)
        pw.check(L.pw_mlp_colsum(_p(b["dY32"]), n, OUT, _p(self.G["b3"]), 1, _s()))
        gemm(b["dY16"], OUT, 1, self.W16["W3"], 1, OUT, n, HIDDEN, OUT, C16=b["dH2_16"], gate=H2, g_m=HIDDEN,
             colsum=self.G["b2"])
        # layer 2
        gemm(H1, 1, HIDDEN, b["dH2_16"], HIDDEN, 1, HIDDEN, HIDDEN, n, C32=self.G["W2"], accumulate=True)
        gemm(b["dH2_16"], HIDDEN, 1, self.W16["W2"], 1, HIDDEN, n, HIDDEN, HIDDEN, C16=b["dH1_16"], gate=H1,
             g_m=HIDDEN, colsum=self.G["b1"])
        # layer 1
        gemm(X16, 1, WIDTH_IN, b["dH1_16"], HIDDEN, 1, WIDTH_IN, HIDDEN, n, C32=self.G["W1"], accumulate=True)
        return self.loss

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        pw.check(_bind().pw_mlp_adam(_p(self.Pf), _p(self.Gf), _p(self.Mf), _p(self.Vf), self.n_par, lr, b1, b2, eps,
                                     self.step, _p(self.W16f), _s()))
        self._sync_t()

    def train_step(self, X16, labels, lr=1e-3):
        Y, H1, H2 = self.forward(X16, keep=True, fresh=False)
        loss = self.backward(X16, H1, H2, Y, labels)
        self.adam_step(lr)
        return loss

    def input_gradient(self, X16, rarity):
        """d score / d input (n x 64 fp32) of the novelty score: the logit
        gradient of the score, propagated back through both ReLU layers."""
        L = _bind()
        n0 = X16.shape[0]
        n = (n0 + 63) // 64 * 64          # the products take multiples of 64 rows: repeat rows to pad
        if n != n0:
            X16 = X16.repeat(((n + n0 - 1) // n0, 1))[:n].contiguous()
        Y, H1, H2 = self.forward(X16, keep=True, fresh=False)
        b = self._buffers(n, X16.device)
        pw.check(L.pw_mlp_score_grad(_p(Y), _p(rarity), n, _p(b["dY16"]), _s()))
        gemm(b["dY16"], OUT, 1, self.W16["W3"], 1, OUT, n, HIDDEN, OUT, C16=b["dH2_16"], gate=H2, g_m=HIDDEN)
        gemm(b["dH2_16"], HIDDEN, 1, self.W16["W2"], 1, HIDDEN, n, HIDDEN, HIDDEN, C16=b["dH1_16"], gate=H1,
             g_m=HIDDEN)
        gemm(b["dH1_16"], HIDDEN, 1, self.W16["W1"], 1, HIDDEN, n, WIDTH_IN, HIDDEN, C32=b["dX"])
        return b["dX"][:n0]


# ------------------------------------------------------------- search loop

def random_masks(seed, offset, n, n_bits, device="cuda"):
    import torch

    out = torch.empty((n, 2), dtype=torch.int64, device=device)
    pw.check(_bind().pw_random_masks(seed, offset, n, n_bits, _p(out), _s()))
    return out


def mutate(parents, n, n_bits, flips, seed):
    import torch

    out = torch.empty((n, 2), dtype=torch.int64, device=parents.device)
    pw.check(_bind().pw_mutate(_p(parents), parents.shape[0], n, n_bits, flips, seed, _p(out), _s()))
    return out


def score(Y, rarity):
    import torch

    out = torch.empty(Y.shape[0], dtype=torch.float32, device=Y.device)
    pw.check(_bind().pw_mlp_score(_p(Y), _p(rarity), Y.shape[0], _p(out), _s()))
    return out


def top_threshold(scores, k, lo, hi, bins=1024):
    """Score above which about k candidates lie: a device histogram of the
    scores, scanned from the top on the host (1024 counts)."""
    import torch

    cnt = torch.zeros(bins, dtype=torch.int32, device=scores.device)
    pw.check(_bind().pw_bin_floats(_p(scores), scores.numel(), lo, hi, bins, _p(cnt), _s()))
    c = cnt.cpu().numpy().view(np.uint32)
    acc = 0
    for b in range(bins - 1, -1, -1):
        acc += int(c[b])
        if acc >= k:
            return lo + (hi - lo) * b / bins
    return -np.inf


def select(scores, cands, threshold, cap):
    import torch

    out = torch.empty((cap, 2), dtype=torch.int64, device=cands.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=cands.device)
    pw.check(_bind().pw_select(_p(scores), _p(cands), cands.shape[0], float(threshold), _p(out), cap, _p(cnt),
                               _s()))
    k = min(int(cnt.item()), cap)
    return out[:k]


def flip_cdf(parents, dX, n_bits, temp=0.25, explore=0.1):
    """Per-parent distribution of the bit to flip (n_parents x 64 cumulative
    probabilities), from the gradient of the novelty score."""
    import torch

    cdf = torch.empty((parents.shape[0], 64), dtype=torch.float32, device=parents.device)
    pw.check(_bind().pw_flip_cdf(_p(parents), _p(dX), dX.shape[1], parents.shape[0], n_bits, temp, explore, _p(cdf),
                                 _s()))
    return cdf


def mutate_guided(parents, dX, n, n_bits, flips, seed, temp=0.25, explore=0.1):
    import torch

    cdf = flip_cdf(parents, dX, n_bits, temp, explore)
    out = torch.empty((n, 2), dtype=torch.int64, device=parents.device)
    pw.check(_bind().pw_mutate_cdf(_p(parents), _p(cdf), parents.shape[0], n, flips, seed, _p(out), _s()))
    return out


def rarity_from_labels(lab):
    """-log of the class frequencies of the six heads over a labelled set
    (counted on the device; 64 numbers come back)."""
    import torch

    cnt = torch.zeros(OUT, dtype=torch.int32, device=lab.device)
    pw.check(_bind().pw_label_counts(_p(lab), lab.shape[0], _p(cnt), _s()))
    return rarity_from_counts(cnt)


def rarity_from_counts(cnt):
    """-log of the class frequencies of the six heads from 64 class counts
    (a device tensor of pw_label_counts)."""
    c = cnt.cpu().numpy().view(np.uint32).astype(np.float64) + 0.5
    r = np.zeros(OUT, dtype=np.float32)
    st = np.concatenate([[0], np.cumsum(HEADS)])
    for h in range(6):
        p = c[st[h]:st[h + 1]] / c[st[h]:st[h + 1]].sum()
        r[st[h]:st[h + 1]] = -np.log(p)
    return r


def rarest_witnesses(hist, archive, k):
    """Masks of the k schemes seen least often (witness = index into the
    device archive of judged masks)."""
    import torch

    h = hist.read()
    ranked = sorted(h.items(), key=lambda kv: kv[1][0])[:k]
    idx = torch.tensor([w for _, (_, w) in ranked], dtype=torch.int64, device=archive.device)
    return archive[idx], len(h)


def run_uniform(tri, d, budget, chunk=1 << 22, seed=1, curve=False):
    """Uniform masks judged by the exact kernel (histogram mode).  With
    curve=True the histogram is read after every chunk (a host round trip,
    so such a run is for the curve, not for timing)."""
    import torch

    nA = (d + 1) * (d + 2) // 2
    hist = pw.Histogram(1 << 14)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    points = []
    while done < budget:
        n = min(chunk, budget - done)
        m = random_masks(seed, done, n, nA)
        m64 = m[:, 0].contiguous() if pw.mask_bytes(d) == 8 else m
        tri.histogram(m64, hist, index_base=done)
        done += n
        if curve:
            points.append((done, len(hist.read())))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"method": "uniform", "evaluations": done, "distinct": len(hist.read()), "gpu_seconds": dt}
    if curve:
        out["full_curve"] = points
        out["curve"] = points[:: max(1, len(points) // 32)] + ([points[-1]] if len(points) > 32 else [])
    return out


def run_search(tri, d, budget, use_net=True, train_n=1 << 24, epochs=1, batch=1 << 16, lr=3e-3, per_round=1 << 22,
               n_elite=4096, temp=0.25, explore=0.1, seed=7, log=None, target=None, time_budget=None,
               online=False, online_batch=1 << 16, targets=()):
    """Mutation search from the witnesses of the rarest schemes seen.

    With use_net, the network (trained first on train_n uniform masks
    labelled by the exact kernel) shapes every mutation: the gradient of its
    novelty score with respect to the parent's signs gives, per bit, the
    first-order gain of flipping it, and flips are drawn in proportion to
    exp(gain / temperature) (pw_flip_cdf, pw_mutate_cdf).  Without it (the ablation)
    the flipped bits are uniform.  Every proposal is judged by the exact
    kernel (histogram mode; witnesses index a device archive of the judged
    masks); the training masks count against the budget.  With `target`,
    the result also holds the seconds (training included) until at least
    that many distinct schemes had been seen; with `time_budget`, the
    number of distinct schemes seen within that many seconds (read at the
    start of each round).  With `online`, the network keeps learning
    during the search: every round it takes one training step on
    `online_batch` of the round's judged mutants (labels from their exact
    codes, which the same pass returns), and the rarity of each feature
    class is re-estimated from every mask judged so far, so the score
    points at classes the search has rarely reached."""
    import torch

    nA = (d + 1) * (d + 2) // 2
    wide = pw.mask_bytes(d) == 16
    archive = torch.empty((budget, 2), dtype=torch.int64, device="cuda")
    hist = pw.Histogram(1 << 14)
    curve = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def judge(masks, at, want_codes=False):
        archive[at:at + masks.shape[0]] = masks
        mm = masks if wide else masks[:, 0].contiguous()
        if want_codes:
            codes = tri.codes_histogram(mm, hist, index_base=at)
            return at + masks.shape[0], codes
        tri.histogram(mm, hist, index_base=at)
        return at + masks.shape[0]

    # labelled data from uniform masks (judged, counted)
    m = random_masks(seed, 0, train_n, nA)
    used = judge(m, 0)
    net = None
    rarity = None
    if use_net:
        codes = tri.batch(m if wide else m[:, 0].contiguous())
        lab = features(codes)
        X = encode(m, train_n, nA)
        net = MLP(n_in=nA, seed=seed)
        for ep in range(epochs):
            for a in range(0, train_n - batch + 1, batch):
                net.train_step(X[a:a + batch], lab[a:a + batch], lr=lr)
        counts = torch.zeros(OUT, dtype=torch.int32, device="cuda")
        pw.check(_bind().pw_label_counts(_p(lab), lab.shape[0], _p(counts), _s()))
        rarity = torch.from_numpy(rarity_from_counts(counts)).cuda()
        del codes, lab, X
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    rnd = 0
    while used < budget:
        rnd += 1
        k = min(per_round, budget - used)
        parents, distinct = rarest_witnesses(hist, archive, n_elite)
        curve.append((used, distinct, round(time.perf_counter() - t0, 4)))
        flips = 1 + rnd % 3
        if use_net:
            np_ = parents.shape[0]
            dX = net.input_gradient(encode(parents, np_, nA), rarity)
            cand = mutate_guided(parents, dX, k, nA, flips, seed * 1000003 + rnd, temp, explore)
        else:
            cand = mutate(parents, k, nA, flips, seed * 1000003 + rnd)
        if use_net and online:
            used, codes = judge(cand, used, want_codes=True)
            lab = features(codes)
            pw.check(_bind().pw_label_counts(_p(lab), lab.shape[0], _p(counts), _s()))
            nb = min(online_batch, (cand.shape[0] // 64) * 64)
            if nb >= 64:
                net.train_step(encode(cand[:nb], nb, nA), lab[:nb], lr=lr)
            rarity = torch.from_numpy(rarity_from_counts(counts)).cuda()
        else:
            used = judge(cand, used)
        if log and rnd % 16 == 0:
            log(f"round {rnd}: {used} evaluations, {distinct} schemes")
    final = len(hist.read())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    curve.append((used, final, round(dt, 4)))
    reach = None
    if target is not None:
        hit = [c for c in curve if c[1] >= target]
        reach = hit[0][2] if hit else None
    reach_k = {}
    for tk in targets:
        hit = [c for c in curve if c[1] >= tk]
        reach_k[int(tk)] = hit[0][2] if hit else None
    within = None
    if time_budget is not None:
        within = max([c[1] for c in curve if c[2] <= time_budget], default=0)
    name = ("learned (online)" if online else "learned") if use_net else "ablation (uniform flips)"
    return {"method": name, "evaluations": used,
            "seconds_to_target": reach, "distinct_within_time_budget": within, "seconds_to": reach_k,
            "distinct": final, "gpu_seconds": dt, "train_seconds": train_s, "rounds": rnd,
            "curve": curve[:: max(1, len(curve) // 32)] + ([curve[-1]] if len(curve) > 32 else [])}
