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
    L.pw_mlp_gemm.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, i32, vp, vp, i64, i32, vp, vp, i64, i32, vp]
    L.pw_mlp_encode.argtypes = [vp, i64, i32, i32, vp, vp]
    L.pw_features.argtypes = [vp, i64, vp, vp]
    L.pw_mlp_softmax_xent.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.pw_mlp_colsum.argtypes = [vp, i64, i32, vp, vp]
    L.pw_mlp_adam.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp, vp]
    L.pw_mlp_score.argtypes = [vp, vp, i64, vp, vp]
    L.pw_to_bf16.argtypes = [vp, i64, vp, vp]
    L.pw_mutate.argtypes = [vp, i64, i64, i32, i32, u64, vp, vp]
    L.pw_select.argtypes = [vp, vp, i64, f32, vp, i64, vp, vp]
    L.pw_random_masks.argtypes = [u64, u64, i64, i32, vp, vp]
    L.pw_bin_floats.argtypes = [vp, i64, f32, f32, i32, vp, vp]
    for n in ("pw_mlp_gemm", "pw_mlp_encode", "pw_features", "pw_mlp_softmax_xent", "pw_mlp_colsum",
              "pw_mlp_adam", "pw_mlp_score", "pw_to_bf16", "pw_mutate", "pw_select",
              "pw_random_masks", "pw_bin_floats"):
        getattr(L, n).restype = i32
    _bound = True
    return L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def gemm(A, a_m, a_k, B, b_k, b_n, M, N, K, C32=None, C16=None, c_m=None, bias=None, gate=None, g_m=0,
         relu=False, accumulate=False):
    """C = A B with element strides (A[m,k] = A[m*a_m + k*a_k], ...)."""
    L = _bind()
    pw.check(L.pw_mlp_gemm(_p(A), a_m, a_k, _p(B), b_k, b_n, M, N, K, _p(bias), _p(gate), g_m, int(relu),
                           _p(C32), _p(C16), N if c_m is None else c_m, int(accumulate), _s()))


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


def to_bf16(t32):
    """fp32 device tensor -> bfloat16 bit patterns (int16 tensor)."""
    import torch

    out = torch.empty(t32.shape, dtype=torch.int16, device=t32.device)
    pw.check(_bind().pw_to_bf16(_p(t32), t32.numel(), _p(out), _s()))
    return out


class MLP:
    """Device parameters: fp32 masters, bf16 copies, Adam moments."""

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
        self.P = {k: torch.from_numpy(v).to(device) for k, v in host.items()}
        self.G = {k: torch.zeros_like(v) for k, v in self.P.items()}
        self.M = {k: torch.zeros_like(v) for k, v in self.P.items()}
        self.V = {k: torch.zeros_like(v) for k, v in self.P.items()}
        self.W16 = {k: torch.empty(self.P[k].shape, dtype=torch.int16, device=device) for k in ("W1", "W2", "W3")}
        self.step = 0
        self.sync16()

    def sync16(self):
        """Refresh the bf16 weight copies from the fp32 masters."""
        L = _bind()
        for k in ("W1", "W2", "W3"):
            pw.check(L.pw_to_bf16(_p(self.P[k]), self.P[k].numel(), _p(self.W16[k]), _s()))

    def load(self, host):
        """Set parameters from host float arrays (tests)."""
        import torch

        for k, v in host.items():
            self.P[k].copy_(torch.from_numpy(np.asarray(v, dtype=np.float32)))
        self.sync16()

    def forward(self, X16, keep=False):
        import torch

        n = X16.shape[0]
        dev = X16.device
        H1 = torch.empty((n, HIDDEN), dtype=torch.int16, device=dev)
        H2 = torch.empty((n, HIDDEN), dtype=torch.int16, device=dev)
        Y = torch.empty((n, OUT), dtype=torch.float32, device=dev)
        gemm(X16, WIDTH_IN, 1, self.W16["W1"], HIDDEN, 1, n, HIDDEN, WIDTH_IN, C16=H1, bias=self.P["b1"], relu=True)
        gemm(H1, HIDDEN, 1, self.W16["W2"], HIDDEN, 1, n, HIDDEN, HIDDEN, C16=H2, bias=self.P["b2"], relu=True)
        gemm(H2, HIDDEN, 1, self.W16["W3"], OUT, 1, n, OUT, HIDDEN, C32=Y, bias=self.P["b3"])
        if keep:
            return Y, H1, H2
        return Y

    def backward(self, X16, H1, H2, Y, labels):
        """Loss and parameter gradients (into self.G) for one batch."""
        import torch

        L = _bind()
        n = X16.shape[0]
        dev = X16.device
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        dY32 = torch.empty((n, OUT), dtype=torch.float32, device=dev)
        dY16 = torch.empty((n, OUT), dtype=torch.int16, device=dev)
        pw.check(L.pw_mlp_softmax_xent(_p(Y), _p(labels), n, _p(dY32), _p(dY16), _p(loss), _s()))
        # layer 3
        gemm(H2, 1, HIDDEN, dY16, OUT, 1, HIDDEN, OUT, n, C32=self.G["W3"])
        pw.check(L.pw_mlp_colsum(_p(dY32), n, OUT, _p(self.G["b3"]), _s()))
        dH2_32 = torch.empty((n, HIDDEN), dtype=torch.float32, device=dev)
        dH2_16 = torch.empty((n, HIDDEN), dtype=torch.int16, device=dev)
        gemm(dY16, OUT, 1, self.W16["W3"], 1, OUT, n, HIDDEN, OUT, C32=dH2_32, C16=dH2_16, gate=H2, g_m=HIDDEN)
        # layer 2
        gemm(H1, 1, HIDDEN, dH2_16, HIDDEN, 1, HIDDEN, HIDDEN, n, C32=self.G["W2"])
        pw.check(L.pw_mlp_colsum(_p(dH2_32), n, HIDDEN, _p(self.G["b2"]), _s()))
        dH1_32 = torch.empty((n, HIDDEN), dtype=torch.float32, device=dev)
        dH1_16 = torch.empty((n, HIDDEN), dtype=torch.int16, device=dev)
        gemm(dH2_16, HIDDEN, 1, self.W16["W2"], 1, HIDDEN, n, HIDDEN, HIDDEN, C32=dH1_32, C16=dH1_16, gate=H1,
             g_m=HIDDEN)
        # layer 1
        gemm(X16, 1, WIDTH_IN, dH1_16, HIDDEN, 1, WIDTH_IN, HIDDEN, n, C32=self.G["W1"])
        pw.check(L.pw_mlp_colsum(_p(dH1_32), n, HIDDEN, _p(self.G["b1"]), _s()))
        return loss

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        L = _bind()
        self.step += 1
        for k in self.P:
            pw.check(L.pw_mlp_adam(_p(self.P[k]), _p(self.G[k]), _p(self.M[k]), _p(self.V[k]), self.P[k].numel(),
                                   lr, b1, b2, eps, self.step, _p(self.W16.get(k)), _s()))

    def train_step(self, X16, labels, lr=1e-3):
        Y, H1, H2 = self.forward(X16, keep=True)
        loss = self.backward(X16, H1, H2, Y, labels)
        self.adam_step(lr)
        return loss


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


def rarest_witnesses(hist, archive, k):
    """Masks of the k schemes seen least often (witness = index into the
    device archive of judged masks)."""
    import torch

    h = hist.read()
    ranked = sorted(h.items(), key=lambda kv: kv[1][0])[:k]
    idx = torch.tensor([w for _, (_, w) in ranked], dtype=torch.int64, device=archive.device)
    return archive[idx], len(h)


def run_uniform(tri, d, budget, chunk=1 << 22, seed=1):
    """Uniform masks judged by the exact kernel (histogram mode)."""
    import torch

    nA = (d + 1) * (d + 2) // 2
    hist = pw.Histogram(1 << 14)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < budget:
        n = min(chunk, budget - done)
        m = random_masks(seed, done, n, nA)
        m64 = m[:, 0].contiguous() if pw.mask_bytes(d) == 8 else m
        tri.histogram(m64, hist, index_base=done)
        done += n
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"method": "uniform", "evaluations": done, "distinct": len(hist.read()), "gpu_seconds": dt}


def run_search(tri, d, budget, use_net=True, train_n=1 << 22, epochs=1, batch=16384, per_round=1 << 21,
               oversample=2, n_elite=4096, seed=7, log=None):
    """Mutation search from the rarest schemes seen, ranked by the network
    (use_net) or at random (the ablation).  Every proposal is judged by the
    exact kernel (histogram mode, witnesses = indices into a device archive
    of the judged masks); the training masks count against the budget."""
    import torch

    nA = (d + 1) * (d + 2) // 2
    wide = pw.mask_bytes(d) == 16
    archive = torch.empty((budget, 2), dtype=torch.int64, device="cuda")
    hist = pw.Histogram(1 << 14)
    curve = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def judge(masks, at):
        archive[at:at + masks.shape[0]] = masks
        tri.histogram(masks if wide else masks[:, 0].contiguous(), hist, index_base=at)
        return at + masks.shape[0]

    # labelled data from uniform masks (judged, counted)
    m = random_masks(seed, 0, train_n, nA)
    used = judge(m, 0)
    net = None
    rarity = None
    score_hi = 1.0
    if use_net:
        codes = tri.batch(m if wide else m[:, 0].contiguous())
        lab = features(codes)
        X = encode(m, train_n, nA)
        net = MLP(n_in=nA, seed=seed)
        for ep in range(epochs):
            for a in range(0, train_n - batch + 1, batch):
                net.train_step(X[a:a + batch], lab[a:a + batch], lr=2e-3)
        labels = lab.cpu().numpy()
        r = np.zeros(OUT, dtype=np.float32)
        st = np.concatenate([[0], np.cumsum(HEADS)])
        for h in range(6):
            p = np.bincount(labels[:, h], minlength=HEADS[h]).astype(np.float64) + 0.5
            p /= p.sum()
            r[st[h]:st[h + 1]] = -np.log(p)
        rarity = torch.from_numpy(r).cuda()
        score_hi = float(sum(r[st[h]:st[h + 1]].max() for h in range(6)))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    rnd = 0
    while used < budget:
        rnd += 1
        k = min(per_round, budget - used)
        parents, distinct = rarest_witnesses(hist, archive, n_elite)
        curve.append((used, distinct))
        cand = mutate(parents, k * (oversample if use_net else 1), nA, 1 + rnd % 3, seed * 1000003 + rnd)
        if use_net:
            Y = net.forward(encode(cand, cand.shape[0], nA))
            sc = score(Y, rarity)
            sel = select(sc, cand, top_threshold(sc, k, 0.0, score_hi), k)
            if sel.shape[0] == 0:
                sel = cand[:k]
        else:
            sel = cand[:k]          # random ranking: the mutants are already in random order
        used = judge(sel, used)
        if log and rnd % 16 == 0:
            log(f"round {rnd}: {used} evaluations, {distinct} schemes")
    final = len(hist.read())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    curve.append((used, final))
    return {"method": "learned" if use_net else "ablation (random ranking)", "evaluations": used,
            "distinct": final, "gpu_seconds": dt, "train_seconds": train_s, "rounds": rnd,
            "curve": curve[:: max(1, len(curve) // 32)] + ([curve[-1]] if len(curve) > 32 else [])}
