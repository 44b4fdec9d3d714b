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
    # gradients computed from the GPU's own activations: compare as norms
    G = R.backward(Xh, from16(H1), from16(H2), dYr, P)
    for k in G:
        g = net.G[k].cpu().numpy().astype(np.float64)
        err = np.linalg.norm(g - G[k]) / (np.linalg.norm(G[k]) + 1e-30)
        assert err <= 2e-2, (k, err)
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
