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
