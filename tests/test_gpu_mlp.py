"""GPU parity of the learned proposal's kernels against oracle/mlp.py.

Tolerances follow from the arithmetic: the GPU multiplies BF16 operands
exactly and accumulates in FP32 (relative error <= K * 2^-24 per dot
product, bounded by the sum of |a||b|); a stored BF16 result adds half an
ulp (2^-9 relative); an FP32 accumulation difference can flip the rounding of
a stored hidden activation by one BF16 ulp (2^-8 relative), which then
propagates through the next products.  Integer work (encoding, feature
classes, mutation) is compared exactly."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import mlp as R
from paper_2604_09221_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2604_09221_amd import learn

    assert torch.cuda.is_available()
    learn._bind()
    return learn


def bits16(x):
    """host float64 values -> bf16 bit patterns (int16) after rounding"""
    f = R.bf16(x).astype(np.float32)
    return torch.from_numpy((f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()


def from16(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K,variant", [(128, 64, 96, "NN"), (64, 512, 64, "NN"), (256, 128, 512, "NT"),
                                           (512, 64, 1024, "TN")])
def test_gemm_variants(L, M, N, K, variant):
    rng = np.random.default_rng(M + N + K)
    A = R.bf16(rng.normal(size=(M, K)))
    B = R.bf16(rng.normal(size=(K, N)))
    bias = rng.normal(size=N).astype(np.float32)
    gate = R.bf16(rng.normal(size=(M, N)))
    if variant == "NN":
        At, a_m, a_k = bits16(A), K, 1
        Bt, b_k, b_n = bits16(B), N, 1
    elif variant == "NT":          # B stored transposed (N x K)
        At, a_m, a_k = bits16(A), K, 1
        Bt, b_k, b_n = bits16(B.T.copy()), 1, K
    else:                          # A stored transposed (K x M)
        At, a_m, a_k = bits16(A.T.copy()), 1, M
        Bt, b_k, b_n = bits16(B), N, 1
    C32 = torch.empty((M, N), dtype=torch.float32, device="cuda")
    C16 = torch.empty((M, N), dtype=torch.int16, device="cuda")
    cs = torch.zeros(N, dtype=torch.float32, device="cuda")
    L.gemm(At, a_m, a_k, Bt, b_k, b_n, M, N, K, C32=C32, C16=C16, bias=torch.from_numpy(bias).cuda(),
           gate=bits16(gate), g_m=N, relu=True, colsum=cs)
    torch.cuda.synchronize()
    want = np.maximum(A @ B + bias, 0.0) * (gate > 0)
    bound = np.abs(A) @ np.abs(B) * K * 2.0 ** -24 + np.abs(bias) * 2.0 ** -24 + 1e-30
    got = C32.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= bound)
    assert np.all(np.abs(from16(C16) - want) <= bound + np.abs(want) * 2.0 ** -8)
    # fused column sums: per-element error plus one rounding per addition
    cbound = bound.sum(axis=0) + (M + 2) * 2.0 ** -24 * np.abs(want).sum(axis=0) + 1e-30
    assert np.all(np.abs(cs.cpu().numpy().astype(np.float64) - want.sum(axis=0)) <= cbound)


@pytest.mark.parametrize("M,N,K,variant,accumulate", [
    (512, 512, 4096, "TN", False),   # weight-gradient shape: K split over blocks, atomic partial sums
    (64, 512, 2048, "TN", True),     # split K on top of an existing C32
    (512, 64, 1024, "TT", False),    # both operands transposed, split K
    (192, 320, 96, "NN", False),     # 64-wide tiles on both axes, ragged against 128
    (128, 192, 64, "GG", True),      # unaligned strides: element-wise staging
])
def test_gemm_plain_fp32(L, M, N, K, variant, accumulate):
    """C32 (+)= A B without epilogue: the path that splits K."""
    rng = np.random.default_rng(7 * M + N + K)
    A = R.bf16(rng.normal(size=(M, K)))
    B = R.bf16(rng.normal(size=(K, N)))
    C0 = rng.normal(size=(M, N)).astype(np.float32)
    if variant == "NN":
        At, a_m, a_k = bits16(A), K, 1
        Bt, b_k, b_n = bits16(B), N, 1
    elif variant == "TN":
        At, a_m, a_k = bits16(A.T.copy()), 1, M
        Bt, b_k, b_n = bits16(B), N, 1
    elif variant == "TT":
        At, a_m, a_k = bits16(A.T.copy()), 1, M
        Bt, b_k, b_n = bits16(B.T.copy()), 1, K
    else:                          # rows padded by 3 elements: no 16-byte alignment
        Ap = np.zeros((M, K + 3)); Ap[:, :K] = A
        Bp = np.zeros((K, N + 3)); Bp[:, :N] = B
        At, a_m, a_k = bits16(Ap), K + 3, 1
        Bt, b_k, b_n = bits16(Bp), N + 3, 1
    C32 = torch.from_numpy(C0.copy()).cuda()
    L.gemm(At, a_m, a_k, Bt, b_k, b_n, M, N, K, C32=C32, accumulate=accumulate)
    torch.cuda.synchronize()
    want = A @ B + (C0.astype(np.float64) if accumulate else 0.0)
    # every partial sum and every atomic addition rounds once in FP32: at
    # most K + (number of splits <= K / 128) roundings, each relative to a
    # value bounded by sum |a||b| (+ |C0|)
    mag = np.abs(A) @ np.abs(B) + (np.abs(C0) if accumulate else 0.0)
    bound = mag * (K + K / 128 + 1) * 2.0 ** -24 + 1e-30
    got = C32.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= bound)


def test_encode_and_features_exact(L):
    d = 8
    E = I.standard_triangulation(d)
    masks = I.random_masks(d, 3, 4096)
    mt = torch.from_numpy(I.masks128(masks)).cuda()
    X = L.encode(mt, len(masks), I.n_points(d))
    assert np.array_equal(from16(X), R.encode(masks, I.n_points(d)))
    codes = oracle.scheme_many(d, E, masks, threads=8)
    ct = torch.from_numpy(codes.view(np.int64)).cuda()
    lab = L.features(ct).cpu().numpy()
    assert np.array_equal(lab, R.features(codes))


def softmax_rel(Y, a, e):
    """Relative error bound of an fp32 softmax probability of head [a, e):
    the shifted logit z = y - max is rounded (relative 2^-24, so exp(z)
    moves by |z| 2^-24) and expf adds at most 4 * 2^-24; the probability
    e_j / sum_i e_i sees that twice (numerator and normaliser), the K - 1
    additions of the normaliser and the division:
    (2 max|z| + 2 K + 10) 2^-24 per row."""
    z = Y[:, a:e] - Y[:, a:e].max(axis=1, keepdims=True)
    return (2 * np.abs(z).max(axis=1, keepdims=True) + 2 * (e - a) + 10) * 2.0 ** -24


def check_softmax_grad(dY32, Y, dY_ref, n):
    """fp32 softmax cross-entropy gradient (p - onehot) / n against the
    float64 one: the probability's error (softmax_rel), the subtraction and
    the division by n (one rounding each)."""
    P = R.head_softmax(Y)
    for h in range(6):
        a, e = R.STARTS[h], R.STARTS[h + 1]
        bound = (P[:, a:e] * softmax_rel(Y, a, e) + 2.0 ** -23) / n
        assert np.all(np.abs(dY32[:, a:e] - dY_ref[:, a:e]) <= bound), h


def check_stored(got16, raw, mag, K):
    """A bf16-stored product against the float64 value of the same
    operands: FP32 accumulation (at most K + 2 roundings of magnitude sum
    |a||b|), then one rounding to bf16 (2^-8 of the value)."""
    acc = mag * (K + 2) * 2.0 ** -24 + 1e-30
    assert np.all(np.abs(got16 - raw) <= acc + 2.0 ** -8 * (np.abs(raw) + acc))


def check_score_grad(dY16, Y, rar):
    """bf16 logit gradient of the novelty score against the float64 one:
    fp32 probabilities (relative error eps_h as in check_softmax_grad), the
    head's expected rarity s_h (eps_h plus K roundings, times sum p |r|),
    then one rounding to bf16."""
    want = R.score_grad(Y, rar)
    P = R.head_softmax(Y)
    for h in range(6):
        a, e = R.STARTS[h], R.STARTS[h + 1]
        K = e - a
        p, r = P[:, a:e], rar[a:e][None, :]
        eps = softmax_rel(Y, a, e)
        sh = (p * r).sum(axis=1, keepdims=True)
        ds = (eps + K * 2.0 ** -24) * (p * np.abs(r)).sum(axis=1, keepdims=True)
        dg = p * (np.abs(r - sh) * (eps + 2.0 ** -22) + ds)
        bound = dg + 2.0 ** -8 * (np.abs(want[:, a:e]) + dg) + 1e-30
        assert np.all(np.abs(dY16[:, a:e] - want[:, a:e]) <= bound), h


def _batch(n=256, seed=0):
    d = 8
    E = I.standard_triangulation(d)
    masks = I.random_masks(d, seed, n)
    codes = oracle.scheme_many(d, E, masks, threads=8)
    return masks, codes


def test_forward_backward_adam_against_oracle(L):
    masks, codes = _batch()
    n = len(masks)
    P = R.init_params(5)
    rng = np.random.default_rng(2)
    for k in P:
        if k.startswith("b"):
            P[k] = rng.normal(scale=0.05, size=P[k].shape).astype(np.float32).astype(np.float64)
    net = L.MLP(seed=0)
    net.load(P)
    X = L.encode(torch.from_numpy(I.masks128(masks)).cuda(), n, 45)
    lab = torch.from_numpy(R.features(codes).astype(np.int32)).cuda()
    Y, H1, H2 = net.forward(X, keep=True)
    loss = net.backward(X, H1, H2, Y, lab)
    torch.cuda.synchronize()
    Xh = R.encode(masks, 45)
    Yr, H1r, H2r = R.forward(Xh, P)
    # hidden activations: at most one bf16 ulp apart
    for g, r in ((H1, H1r), (H2, H2r)):
        gh = from16(g)
        assert np.all(np.abs(gh - r) <= np.abs(r) * 2.0 ** -7 + 1e-6)
    Yg = Y.cpu().numpy().astype(np.float64)
    scale = np.abs(H2r) @ np.abs(R.bf16(P["W3"]))
    assert np.all(np.abs(Yg - Yr) <= scale * 2.0 ** -6 + 1e-5)
    lr_, dYr = R.softmax_xent(Yg, R.features(codes))
    assert abs(loss.item() - lr_) <= 1e-4 * abs(lr_)
    # every gradient element against the oracle, each layer fed the values
    # the GPU stored for its inputs (activations, dY, dH2, dH1)
    b = net._buf[n]
    dY32 = b["dY32"].cpu().numpy().astype(np.float64)
    check_softmax_grad(dY32, Yg, dYr, n)
    dY16, dH2, dH1 = from16(b["dY16"]), from16(b["dH2_16"]), from16(b["dH1_16"])
    assert np.array_equal(dY16, R.bf16(dY32))              # the bf16 copy of the same fp32 values
    H1g, H2g = from16(H1), from16(H2)
    st = {}
    G = R.backward(Xh, H1g, H2g, dY32, P, given={"dY16": dY16, "dH2": dH2, "dH1": dH1}, stages=st)
    W = {k: R.bf16(P[k]) for k in ("W1", "W2", "W3")}
    # stored hidden gradients: the fp32 product (K = 64, 512) rounded once to bf16
    check_stored(dH2, st["dH2_raw"], (np.abs(dY16) @ np.abs(W["W3"]).T) * (H2g > 0), 64)
    check_stored(dH1, st["dH1_raw"], (np.abs(dH2) @ np.abs(W["W2"]).T) * (H1g > 0), 512)
    # weight gradients: K = n rows, split over blocks and added atomically
    mags = {"W3": np.abs(H2g).T @ np.abs(dY16), "W2": np.abs(H1g).T @ np.abs(dH2),
            "W1": np.abs(Xh).T @ np.abs(dH1)}
    for k, mag in mags.items():
        g = net.G[k].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(g - G[k]) <= mag * (n + n / 128 + 2) * 2.0 ** -24 + 1e-30), k
    # bias gradients: b3 = column sums of dY (fp32, 256-row blocks + atomics);
    # b2, b1 = column sums of the fp32 products before their bf16 rounding
    colmag = {"b3": (np.abs(dY32).sum(axis=0), 0.0),
              "b2": ((np.abs(dY16) @ np.abs(W["W3"]).T * (H2g > 0)).sum(axis=0), 64),
              "b1": ((np.abs(dH2) @ np.abs(W["W2"]).T * (H1g > 0)).sum(axis=0), 512)}
    for k, (mag, K) in colmag.items():
        g = net.G[k].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(g - G[k]) <= mag * (n + K + 4) * 2.0 ** -24 + 1e-30), k
    # one Adam step on the same gradients
    before = {k: net.P[k].cpu().numpy().astype(np.float64) for k in net.P}
    grads = {k: net.G[k].cpu().numpy().astype(np.float64) for k in net.P}
    net.adam_step(lr=1e-3)
    torch.cuda.synchronize()
    for k in net.P:
        w, _, _ = R.adam(before[k], grads[k], np.zeros_like(before[k]), np.zeros_like(before[k]), 1, lr=1e-3)
        assert np.allclose(net.P[k].cpu().numpy(), w, rtol=1e-5, atol=1e-6), k


def test_training_reduces_loss(L):
    """A few hundred Adam steps on kernel-labelled masks: the loss falls well
    below its initial value and below the entropy of the label marginals
    (what a network ignoring its input could reach)."""
    from paper_2604_09221_amd import patchwork as pw

    d = 8
    tri = pw.Triangulation(d, I.standard_triangulation(d))
    n = 1 << 16
    masks = I.random_masks(d, 11, n)
    mt = torch.from_numpy(I.masks128(masks)).cuda()
    codes = tri.batch(pw.mask_tensor(masks, d))
    lab = L.features(codes)
    X = L.encode(mt, n, 45)
    net = L.MLP(seed=1)
    bs = 1024
    losses = []
    for step in range(300):
        a = (step * bs) % n
        losses.append(net.train_step(X[a:a + bs], lab[a:a + bs], lr=1e-3).item())
    labels = lab.cpu().numpy()
    marginal = 0.0
    for h in range(6):
        p = np.bincount(labels[:, h], minlength=R.HEADS[h]) / n
        marginal += -(p[p > 0] * np.log(p[p > 0])).sum()
    assert np.mean(losses[-20:]) < 0.9 * losses[0]
    assert np.mean(losses[-20:]) < marginal


def test_score_and_score_grad_against_oracle(L):
    """pw_mlp_score and pw_mlp_score_grad on logits of several scales
    (including heads dominated by one logit) against the float64 oracle."""
    rng = np.random.default_rng(21)
    n = 4096
    Y = (rng.normal(size=(n, 64)) * rng.choice([0.1, 1.0, 4.0, 12.0], size=(n, 1))).astype(np.float32)
    rar = rng.uniform(0.0, 8.0, size=64).astype(np.float32)
    Yt, rt = torch.from_numpy(Y).cuda(), torch.from_numpy(rar).cuda()
    sc = L.score(Yt, rt).cpu().numpy().astype(np.float64)
    dY = torch.empty((n, 64), dtype=torch.int16, device="cuda")
    from paper_2604_09221_amd import patchwork as pwb
    pwb.check(L._bind().pw_mlp_score_grad(L._p(Yt), L._p(rt), n, L._p(dY), L._s()))
    torch.cuda.synchronize()
    Y64, r64 = Y.astype(np.float64), rar.astype(np.float64)
    want = R.score(Y64, r64)
    P = R.head_softmax(Y64)
    bound = np.zeros(n)
    for h in range(6):
        # s_h = acc / z: the probabilities' error plus the K roundings of acc
        a, e = R.STARTS[h], R.STARTS[h + 1]
        eps = softmax_rel(Y64, a, e)[:, 0] + (e - a) * 2.0 ** -24
        bound += eps * (P[:, a:e] * np.abs(r64[a:e])).sum(axis=1)
    bound += 6 * 2.0 ** -24 * np.abs(want)
    assert np.all(np.abs(sc - want) <= bound)
    check_score_grad(from16(dY), Y64, r64)


def test_input_gradient_against_oracle(L):
    """MLP.input_gradient (forward, score gradient, three backward products)
    element by element: each stage against the oracle fed the GPU's stored
    values of that stage's inputs."""
    masks, codes = _batch(n=200, seed=4)            # 200 rows: padded to 256 by repetition
    n0 = len(masks)
    P = R.init_params(6)
    rng = np.random.default_rng(3)
    for k in P:
        if k.startswith("b"):
            P[k] = rng.normal(scale=0.05, size=P[k].shape).astype(np.float32).astype(np.float64)
    net = L.MLP(seed=0)
    net.load(P)
    rar = rng.uniform(0.0, 6.0, size=64).astype(np.float32)
    X = L.encode(torch.from_numpy(I.masks128(masks)).cuda(), n0, 45)
    dX = net.input_gradient(X, torch.from_numpy(rar).cuda()).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    n = 256
    b = net._buf[n]
    Yg = b["Y"].cpu().numpy().astype(np.float64)
    H1g, H2g = from16(b["H1"]), from16(b["H2"])
    dY16, dH2, dH1 = from16(b["dY16"]), from16(b["dH2_16"]), from16(b["dH1_16"])
    # the forward pass of the padded batch is the forward pass of its rows
    Xh = R.encode(masks, 45)
    Xpad = np.concatenate([Xh, Xh[:n - n0]])
    Yr, H1r, H2r = R.forward(Xpad, P)
    assert np.all(np.abs(H1g - H1r) <= np.abs(H1r) * 2.0 ** -7 + 1e-6)
    assert np.all(np.abs(H2g - H2r) <= np.abs(H2r) * 2.0 ** -7 + 1e-6)
    check_score_grad(dY16, Yg, rar.astype(np.float64))
    st = {}
    want = R.input_gradient(Yg, H1g, H2g, P, rar.astype(np.float64), given={"dY16": dY16, "dH2": dH2, "dH1": dH1},
                            stages=st)
    W = {k: R.bf16(P[k]) for k in ("W1", "W2", "W3")}
    check_stored(dH2, st["dH2_raw"], (np.abs(dY16) @ np.abs(W["W3"]).T) * (H2g > 0), 64)
    check_stored(dH1, st["dH1_raw"], (np.abs(dH2) @ np.abs(W["W2"]).T) * (H1g > 0), 512)
    mag = np.abs(dH1) @ np.abs(W["W1"]).T
    assert np.all(np.abs(dX - want[:n0]) <= mag[:n0] * 514 * 2.0 ** -24 + 1e-30)
    assert np.all(dX[:, 45:] == 0.0)                 # padding columns of W1 are zero


def test_mutation_kernels_exact(L):
    """pw_mutate and pw_mutate_cdf draw the same bits as the oracle's
    counter-based generator (bit-exact), and pw_flip_cdf's table matches
    the oracle's formula."""
    rng = np.random.default_rng(31)
    nb, n_par, n = 45, 64, 4096
    par = np.zeros((n_par, 2), dtype=np.uint64)
    par[:, 0] = rng.integers(0, 1 << 45, size=n_par, dtype=np.uint64) & ~np.uint64(1)
    pt = torch.from_numpy(par.view(np.int64)).cuda()
    for flips, seed in ((1, 5), (3, 2**63 + 12345)):
        got = L.mutate(pt, n, nb, flips, seed).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, R.mutate(par, n, nb, flips, seed))
    dX = rng.normal(size=(n_par, 64)).astype(np.float32)
    dX[0] = 0.0                                       # a parent with no gradient: uniform flips
    cdf = L.flip_cdf(pt, torch.from_numpy(dX).cuda(), nb, 0.3, 0.1)
    c = cdf.cpu().numpy()
    assert np.allclose(c.astype(np.float64), R.flip_cdf(par, dX.astype(np.float64), nb, 0.3, 0.1), atol=2e-6, rtol=0)
    from paper_2604_09221_amd import patchwork as pwb
    for flips, seed in ((1, 99), (2, 7)):
        out = torch.empty((n, 2), dtype=torch.int64, device="cuda")
        pwb.check(L._bind().pw_mutate_cdf(L._p(pt), L._p(cdf), n_par, n, flips, seed, L._p(out), L._s()))
        got = out.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, R.mutate_cdf(par, c, n, flips, seed))


def test_random_masks_bins_and_select_exact(L):
    """pw_random_masks is the SplitMix64 stream (two outputs per mask);
    pw_bin_floats and pw_select against the oracle's binary32 rules."""
    for nb, seed, off in ((45, 3, 0), (91, 8, 1000)):
        got = L.random_masks(seed, off, 5000, nb).cpu().numpy().view(np.uint64)
        z = I.splitmix64(seed, 2 * 5000, offset=2 * off).reshape(-1, 2)
        lo = z[:, 0] & np.uint64((1 << min(nb, 64)) - 1 if nb < 64 else 2**64 - 1) & ~np.uint64(1)
        hi = z[:, 1] & np.uint64((1 << (nb - 64)) - 1) if nb > 64 else np.zeros(len(z), dtype=np.uint64)
        assert np.array_equal(got[:, 0], lo) and np.array_equal(got[:, 1], hi)
    rng = np.random.default_rng(41)
    x = np.concatenate([rng.normal(2.0, 3.0, size=100000), [-50.0, 50.0, 8.0, -4.0]]).astype(np.float32)
    for lo_, hi_, bins in ((-4.0, 8.0, 1024), (0.5, 3.25, 77)):
        cnt = torch.zeros(bins, dtype=torch.int32, device="cuda")
        from paper_2604_09221_amd import patchwork as pwb
        pwb.check(L._bind().pw_bin_floats(L._p(torch.from_numpy(x).cuda()), len(x), lo_, hi_, bins, L._p(cnt),
                                          L._s()))
        assert np.array_equal(cnt.cpu().numpy().astype(np.int64), R.bin_floats(x, lo_, hi_, bins))
    cand = rng.integers(0, 2**63, size=(len(x), 2), dtype=np.int64)
    for thr, cap in ((2.0, 1 << 17), (5.0, 1000)):
        out = L.select(torch.from_numpy(x).cuda(), torch.from_numpy(cand).cuda(), thr, cap).cpu().numpy()
        kept, count = R.select(x, cand.view(np.uint64), thr)
        assert len(out) == min(count, cap)
        got = {tuple(r) for r in out.view(np.uint64).tolist()}
        want = {tuple(r) for r in kept.tolist()}
        assert got <= want and (len(got) == len(want) or len(got) == cap)


@pytest.mark.parametrize("rows,cols", [(64, 512), (512, 512), (512, 64), (33, 70), (1, 5)])
def test_bf16_transpose_exact(rows, cols):
    from paper_2604_09221_amd import learn as Lr

    rng = np.random.default_rng(rows * 1000 + cols)
    x = rng.integers(-32768, 32767, size=(rows, cols), dtype=np.int16)
    got = Lr.transpose16(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), x.T)


def test_forward_uses_transposed_weights_consistently():
    """The forward products read the [out][in] copies of the weights; after
    an Adam step those copies equal the transposes of the updated bf16
    weights."""
    from paper_2604_09221_amd import learn as Lr

    net = Lr.MLP(n_in=45, seed=3)
    X = Lr.encode(torch.from_numpy(I.masks128(I.random_masks(8, 4, 128))).cuda().view(-1, 2), 128, 45)
    lab = Lr.features(torch.zeros((128, 2), dtype=torch.int64, device="cuda") + 6)
    net.train_step(X, lab, lr=1e-2)
    torch.cuda.synchronize()
    for k, t in net.W16T.items():
        assert torch.equal(t, net.W16[k].t().contiguous()), k
