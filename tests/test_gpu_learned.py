"""What the trained network adds to the proposal search.

The network is trained on the GPU (project kernels) on masks labelled by the
exact kernel.  Mutants of the rarest schemes' witnesses are then drawn two
ways: with flips guided by the gradient of the network's novelty score (the
learned proposal) and with uniform flips (the ablation).  Every mutant is
judged by the exact kernel.  The guided mutants' true feature rarity must
beat the uniform mutants', and so must their share of schemes never seen in
the training set.  A second check ranks uniform mutants by the network's
score: its top 10% must be rarer than a random 10%."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mlp as R
from paper_2604_09221_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    from paper_2604_09221_amd import learn as Lr
    from paper_2604_09221_amd import patchwork as pw

    d, nA = 8, 45
    tri = pw.Triangulation(d, I.standard_triangulation(d))
    n = 1 << 19
    m = Lr.random_masks(3, 0, n, nA)
    codes = tri.batch(m[:, 0].contiguous())
    lab = Lr.features(codes)
    X = Lr.encode(m, n, nA)
    net = Lr.MLP(n_in=nA, seed=4)
    for ep in range(2):
        for a in range(0, n, 4096):
            net.train_step(X[a:a + 4096], lab[a:a + 4096], lr=1e-3)
    rar = Lr.rarity_from_labels(lab)
    hist = pw.Histogram(1 << 12)
    tri.histogram(m[:, 0].contiguous(), hist)
    seen = set(hist.read())
    parents, _ = Lr.rarest_witnesses(hist, m, 2048)
    return Lr, pw, tri, net, rar, seen, parents, nA


def _judge(Lr, tri, cand, rar, seen):
    st = np.concatenate([[0], np.cumsum(Lr.HEADS)])
    codes = tri.batch(cand[:, 0].contiguous())
    tl = Lr.features(codes).cpu().numpy()
    rarity = sum(rar[st[h] + tl[:, h]] for h in range(6))
    c = codes.cpu().numpy().view(np.uint64)
    novel = np.array([(int(a) | (int(b) << 64)) not in seen for a, b in c])
    return rarity, novel


def test_label_counts_match_host(trained):
    Lr, pw, tri, net, rar, seen, parents, nA = trained
    m = Lr.random_masks(5, 0, 1 << 14, nA)
    lab = Lr.features(tri.batch(m[:, 0].contiguous()))
    got = Lr.rarity_from_labels(lab)
    labels = lab.cpu().numpy()
    st = np.concatenate([[0], np.cumsum(Lr.HEADS)])
    for h in range(6):
        c = np.bincount(labels[:, h], minlength=Lr.HEADS[h]).astype(np.float64) + 0.5
        assert np.allclose(got[st[h]:st[h + 1]], -np.log(c / c.sum()), rtol=1e-6)


def test_guided_mutation_beats_uniform_flips(trained):
    Lr, pw, tri, net, rar, seen, parents, nA = trained
    n = 1 << 16
    dX = net.input_gradient(Lr.encode(parents, parents.shape[0], nA), torch.from_numpy(rar).cuda())
    assert torch.isfinite(dX).all()
    guided = Lr.mutate_guided(parents, dX, n, nA, 2, 12345)
    uniform = Lr.mutate(parents, n, nA, 2, 12345)
    # guided mutants differ from their parents in at most 2 bits, bit 0 kept
    p = parents.repeat((n + parents.shape[0] - 1) // parents.shape[0], 1)[:n]
    diff = (guided ^ p).cpu().numpy().view(np.uint64)
    flips = np.array([bin(int(a)).count("1") + bin(int(b)).count("1") for a, b in diff])
    assert flips.max() <= 2 and not (diff[:, 0] & np.uint64(1)).any()
    rg, ng = _judge(Lr, tri, guided, rar, seen)
    ru, nu = _judge(Lr, tri, uniform, rar, seen)
    assert rg.mean() > ru.mean()
    assert ng.mean() >= nu.mean()
    assert tri.errors() == 0


def test_network_ranking_beats_random_ranking(trained):
    Lr, pw, tri, net, rar, seen, parents, nA = trained
    cand = Lr.mutate(parents, 1 << 16, nA, 2, 777)
    sc = Lr.score(net.forward(Lr.encode(cand, cand.shape[0], nA)), torch.from_numpy(rar).cuda()).cpu().numpy()
    true_rarity, novel = _judge(Lr, tri, cand, rar, seen)
    k = len(sc) // 10
    top = np.argsort(-sc)[:k]
    rnd = np.random.default_rng(0).choice(len(sc), k, replace=False)
    assert true_rarity[top].mean() > 1.1 * true_rarity[rnd].mean()
    assert novel[top].mean() >= novel[rnd].mean()


def test_flip_distribution_and_sampling():
    """pw_flip_cdf against the oracle's table, and pw_mutate_cdf's draws
    against the distribution (one parent, 2^20 single flips, 5 sigma)."""
    from paper_2604_09221_amd import learn as Lr

    rng = np.random.default_rng(5)
    n_bits, n_par = 45, 64
    par = np.zeros((n_par, 2), dtype=np.uint64)
    par[:, 0] = rng.integers(0, 1 << 45, size=n_par, dtype=np.uint64) & ~np.uint64(1)
    dX = rng.normal(size=(n_par, 64)).astype(np.float32)
    temp, explore = 0.3, 0.1
    pt = torch.from_numpy(par.view(np.int64)).cuda()
    cdf = Lr.flip_cdf(pt, torch.from_numpy(dX).cuda(), n_bits, temp, explore).cpu().numpy().astype(np.float64)
    want = R.flip_cdf(par, dX.astype(np.float64), n_bits, temp, explore)
    assert np.allclose(cdf, want, atol=2e-6, rtol=0)
    n = 1 << 20
    one = pt[:1].contiguous()
    out = Lr.mutate_guided(one, torch.from_numpy(dX[:1]).cuda(), n, n_bits, 1, 99, temp, explore)
    diff = (out.cpu().numpy().view(np.uint64)[:, 0] ^ par[0, 0])
    bits = np.log2(diff.astype(np.float64)).round().astype(int)
    freq = np.bincount(bits, minlength=64)[:64] / n
    prob = np.concatenate([[0.0], np.diff(cdf[0][:n_bits]), [1.0 - cdf[0][n_bits - 1]]])[:n_bits]
    assert freq[0] == 0 and freq[n_bits:].sum() == 0
    sigma = np.sqrt(prob * (1 - prob) / n)
    assert np.all(np.abs(freq[:n_bits] - prob) <= 5 * sigma + 1e-6)
