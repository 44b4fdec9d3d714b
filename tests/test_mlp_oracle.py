"""Pins of the MLP oracle (oracle/mlp.py) against closed forms and numeric
derivatives, so that the GPU training kernels are compared with something
other than a retyped formula."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import mlp as R


def test_bf16_rounding_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa
    assert R.bf16(1.0 + 2.0 ** -8) == 1.0
    assert R.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert R.bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7
    assert R.bf16(-3.0) == -3.0
    assert R.bf16(0.1) == 0.10009765625          # nearest representable to 0.1
    x = np.random.default_rng(0).normal(size=1000)
    assert np.all(np.abs(R.bf16(x) - x) <= np.abs(x) * 2.0 ** -8 + 1e-40)


def test_loss_at_zero_logits_is_sum_of_log_classes():
    Y = np.zeros((7, 64))
    labels = np.zeros((7, 6), dtype=np.int64)
    loss, dY = R.softmax_xent(Y, labels)
    assert np.isclose(loss, sum(np.log(h) for h in R.HEADS))
    # each head's gradient sums to zero per sample
    for h in range(6):
        assert np.allclose(dY[:, R.STARTS[h]:R.STARTS[h + 1]].sum(axis=1), 0.0)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    n = 6
    X = np.where(rng.random((n, 64)) < 0.5, -1.0, 1.0)
    X[:, 45:] = 0.0
    P = R.init_params(3)
    for k in P:
        if k.startswith("b"):
            P[k] = rng.normal(scale=0.1, size=P[k].shape)
    labels = np.stack([rng.integers(0, h, size=n) for h in R.HEADS], axis=1)

    def f(P):
        Y, _, _ = R.forward(X, P, emulate_bf16=False)
        return R.softmax_xent(Y, labels)[0]

    Y, H1, H2 = R.forward(X, P, emulate_bf16=False)
    _, dY = R.softmax_xent(Y, labels)
    G = R.backward(X, H1, H2, dY, P, emulate_bf16=False)
    eps = 1e-6
    for name, idx in [("W1", (3, 10)), ("W1", (44, 500)), ("b1", (7,)), ("W2", (100, 200)), ("b2", (300,)),
                      ("W3", (17, 5)), ("W3", (400, 63)), ("b3", (30,))]:
        Pp = {k: v.copy() for k, v in P.items()}
        Pm = {k: v.copy() for k, v in P.items()}
        Pp[name][idx] += eps
        Pm[name][idx] -= eps
        num = (f(Pp) - f(Pm)) / (2 * eps)
        assert abs(num - G[name][idx]) <= 1e-6 + 1e-4 * abs(num), (name, idx, num, G[name][idx])


def test_adam_first_steps_closed_form():
    """On f(w) = w^2 / 2 the first Adam step moves w by lr in the direction
    of -g (m_hat / sqrt(v_hat) = sign(g) when the moments start at 0)."""
    w = np.array([2.0, -3.0])
    m = np.zeros(2)
    v = np.zeros(2)
    w1, m, v = R.adam(w, w, m, v, 1, lr=0.01)
    assert np.allclose(w1, w - 0.01 * np.sign(w), atol=1e-9)
    w2, m, v = R.adam(w1, w1, m, v, 2, lr=0.01)
    mh = (0.9 * 0.1 * w + 0.1 * w1) / (1 - 0.81)
    vh = (0.999 * 0.001 * w * w + 0.001 * w1 * w1) / (1 - 0.999 ** 2)
    assert np.allclose(w2, w1 - 0.01 * mh / (np.sqrt(vh) + 1e-8))


def test_features_of_known_schemes():
    J = oracle.J_BIT
    harnack8 = oracle.code_from_forest([[[]] * 3] + [[]] * 18, False)    # <1<3> + 18>, d = 8
    nest = oracle.code_from_forest([[[[[]]]]], False)                   # <1<1<1<1>>>>
    codes = np.array([[harnack8 & (2**64 - 1), harnack8 >> 64], [nest, 0], [1, J >> 64], [6, 0]], dtype=np.uint64)
    f = R.features(codes)
    assert f[0].tolist() == [22, 2, 8, 3, 0, 0]
    assert f[1].tolist() == [4, 4, 1, 1, 1, 1]
    assert f[2].tolist() == [0, 0, 0, 0, 0, 0]
    assert f[3].tolist() == [1, 1, 1, 0, 0, 0]


def test_encode():
    m = np.array([[0b101, 0]], dtype=np.uint64)
    X = R.encode(m, 45)
    assert X[0, :4].tolist() == [-1, 1, -1, 1] and X[0, 44] == 1 and X[0, 45] == 0


# ------------------------------------------------------- novelty score pins

def _rand_logits(n, seed, scale=2.0):
    return np.random.default_rng(seed).normal(scale=scale, size=(n, 64))


def test_score_at_equal_logits_is_mean_rarity_per_head():
    """Equal logits within a head make the softmax uniform, so the score is
    the sum over heads of the mean rarity of the head's classes."""
    rar = np.random.default_rng(3).uniform(0, 5, size=64)
    Y = np.zeros((4, 64))
    for h in range(6):
        Y[:, R.STARTS[h]:R.STARTS[h + 1]] = 0.7 * h - 1.0     # any constant per head
    want = sum(rar[R.STARTS[h]:R.STARTS[h + 1]].mean() for h in range(6))
    assert np.allclose(R.score(Y, rar), want, rtol=1e-14)


def test_score_one_hot_limit():
    """A logit 60 above the rest of its head puts (up to e^-60) all the mass
    on that class: the score is the sum of the chosen classes' rarities."""
    rng = np.random.default_rng(4)
    rar = rng.uniform(0, 5, size=64)
    Y = rng.normal(size=(8, 64))
    want = np.zeros(8)
    for k in range(8):
        for h in range(6):
            j = R.STARTS[h] + int(rng.integers(0, R.HEADS[h]))
            Y[k, j] = Y[k, R.STARTS[h]:R.STARTS[h + 1]].max() + 60.0
            want[k] += rar[j]
    assert np.allclose(R.score(Y, rar), want, atol=1e-20 + 5 * 23 * np.exp(-59))


def test_score_grad_matches_finite_differences():
    rng = np.random.default_rng(5)
    rar = rng.uniform(0, 5, size=64)
    Y = _rand_logits(5, 6)
    G = R.score_grad(Y, rar)
    eps = 1e-6
    for k in range(5):
        for j in (0, 7, 22, 23, 27, 30, 45, 54, 63):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[k, j] += eps
            Ym[k, j] -= eps
            num = (R.score(Yp[k:k + 1], rar)[0] - R.score(Ym[k:k + 1], rar)[0]) / (2 * eps)
            assert abs(num - G[k, j]) <= 1e-8 + 1e-6 * abs(num), (k, j, num, G[k, j])


def test_score_grad_sums_to_zero_per_head():
    """Adding a constant to a head's logits leaves its softmax, hence the
    score, unchanged: the gradient entries of each head sum to zero."""
    rar = np.random.default_rng(7).uniform(0, 5, size=64)
    G = R.score_grad(_rand_logits(16, 8), rar)
    for h in range(6):
        assert np.allclose(G[:, R.STARTS[h]:R.STARTS[h + 1]].sum(axis=1), 0.0, atol=1e-13)


def test_input_gradient_matches_finite_differences():
    """d score(forward(X)) / d X in float64 against central differences of
    the composed function (X treated as continuous)."""
    rng = np.random.default_rng(9)
    P = R.init_params(2)
    for k in P:
        if k.startswith("b"):
            P[k] = rng.normal(scale=0.1, size=P[k].shape)
    rar = rng.uniform(0, 5, size=64)
    X = np.where(rng.random((3, 64)) < 0.5, -1.0, 1.0)
    X[:, 45:] = 0.0

    def s(Xk):
        return R.score(R.forward(Xk, P, emulate_bf16=False)[0], rar)

    Y, H1, H2 = R.forward(X, P, emulate_bf16=False)
    dX = R.input_gradient(Y, H1, H2, P, rar, emulate_bf16=False)
    eps = 1e-6
    for k in range(3):
        for j in (0, 1, 13, 30, 44):
            Xp, Xm = X.copy(), X.copy()
            Xp[k, j] += eps
            Xm[k, j] -= eps
            num = (s(Xp)[k] - s(Xm)[k]) / (2 * eps)
            assert abs(num - dX[k, j]) <= 1e-7 + 1e-5 * abs(num), (k, j, num, dX[k, j])


def test_bf16_backward_within_rounding_bound_of_float64():
    """The bfloat16-emulating backward pass differs from the float64 one only
    by the roundings it makes: each stored operand moves by at most 2^-8 of
    its magnitude (bfloat16 keeps 8 significant bits), so a gradient entry moves by at most (number of rounded
    operands on its path) * 2^-8 (+ second order) of the sum of the
    magnitudes of the terms that make it up."""
    rng = np.random.default_rng(10)
    n = 32
    P = R.init_params(4)
    X = np.where(rng.random((n, 64)) < 0.5, -1.0, 1.0)
    X[:, 45:] = 0.0
    Y, H1, H2 = R.forward(X, P, emulate_bf16=False)
    labels = np.stack([rng.integers(0, h, size=n) for h in R.HEADS], axis=1)
    _, dY = R.softmax_xent(Y, labels)
    G64 = R.backward(X, H1, H2, dY, P, emulate_bf16=False)
    Gbf = R.backward(X, H1, H2, dY, P, emulate_bf16=True)
    u = 2.0 ** -8 * 1.01
    aW3, aW2, aW1 = np.abs(P["W3"]), np.abs(P["W2"]), np.abs(P["W1"])
    mdH2 = (np.abs(dY) @ aW3.T) * (H2 > 0)            # magnitude of the terms of dH2
    mdH1 = (mdH2 @ aW2.T) * (H1 > 0)
    bounds = {"W3": np.abs(H2).T @ np.abs(dY) * u, "b3": np.zeros(64),
              "W2": np.abs(H1).T @ mdH2 * 4 * u, "b2": mdH2.sum(axis=0) * 2 * u,
              "W1": np.abs(X).T @ mdH1 * 6 * u, "b1": mdH1.sum(axis=0) * 4 * u}
    for k in G64:
        assert np.all(np.abs(Gbf[k] - G64[k]) <= bounds[k] + 1e-300), k
        assert np.any(Gbf[k] != G64[k]) or k == "b3"       # the roundings do happen


# ------------------------------------------------------- proposal sampling pins

def test_splitmix_published_outputs():
    """The first three outputs of SplitMix64 seeded with 0 (the generator's
    reference implementation)."""
    g = 0x9E3779B97F4A7C15
    assert [R.splitmix_mix(i * g % 2**64) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                                 0x06C45D188009454F]


def test_mutate_flips_are_uniform_and_spare_bit0():
    par = np.array([[0, 0], [0b1010, 1 << 3]], dtype=np.uint64)
    n, nb = 40000, 45
    out = R.mutate(par, n, nb, 1, 5)
    diff = out ^ par[np.arange(n) % 2]
    assert not (diff[:, 1]).any() and not (diff[:, 0] & np.uint64(1)).any()
    bits = np.log2(diff[:, 0].astype(np.float64)).round().astype(int)
    freq = np.bincount(bits, minlength=nb)
    assert freq[0] == 0 and freq[1:].sum() == n
    e = n / (nb - 1)
    chi2 = ((freq[1:] - e) ** 2 / e).sum()
    assert chi2 < 44 + 6 * np.sqrt(2 * 44)                # 44 degrees of freedom, 6 sigma


def test_flip_cdf_special_cases():
    par = np.zeros((2, 2), dtype=np.uint64)
    nb = 45
    # zero gradient: every gain is zero, the distribution is uniform
    c = R.flip_cdf(par, np.zeros((2, 64)), nb, 0.3, 0.1)
    assert np.allclose(c[0, :nb - 1], np.arange(nb - 1) / (nb - 1)) and np.all(c[:, nb - 1:] == 1.0)
    # one dominant gain at a tiny temperature: that bit takes (1 - explore) + explore / (nb - 1)
    dX = np.zeros((2, 64))
    dX[0, 17] = -1.0                       # x = +1 ('+'), gain = -2 * dX = 2 > 0
    c = R.flip_cdf(par, dX, nb, 1e-3, 0.1)
    p = np.diff(np.concatenate([c[0, :nb - 1], [1.0]]))
    assert np.isclose(p[16], 0.9 + 0.1 / (nb - 1)) and np.allclose(np.delete(p, 16), 0.1 / (nb - 1))


def test_mutate_cdf_follows_the_table():
    rng = np.random.default_rng(12)
    nb = 45
    par = np.zeros((1, 2), dtype=np.uint64)
    c = R.flip_cdf(par, rng.normal(size=(1, 64)), nb, 0.3, 0.1)
    n = 60000
    out = R.mutate_cdf(par, c, n, 1, 77)
    bits = np.log2(out[:, 0].astype(np.float64)).round().astype(int)
    freq = np.bincount(bits, minlength=64)[:64] / n
    prob = np.diff(np.concatenate([c[0, :nb - 1], [1.0]]))
    assert freq[0] == 0 and freq[nb:].sum() == 0
    sigma = np.sqrt(prob * (1 - prob) / n)
    assert np.all(np.abs(freq[1:nb] - prob) <= 5 * sigma + 1e-9)


def test_bin_floats_centres_and_clamping():
    lo, hi, bins = -2.0, 6.0, 16
    w = (hi - lo) / bins
    x = np.concatenate([lo + (np.arange(bins) + 0.5) * w, [-100.0, 100.0, hi]])
    c = R.bin_floats(x, lo, hi, bins)
    want = np.ones(bins, dtype=np.int64)
    want[0] += 1
    want[-1] += 2
    assert np.array_equal(c, want)


def test_select_keeps_strictly_greater():
    cand = np.arange(10, dtype=np.uint64).reshape(5, 2)
    kept, n = R.select([0.5, 1.0, 1.5, 1.0, 2.0], cand, 1.0)
    assert n == 2 and kept.tolist() == [[4, 5], [8, 9]]
