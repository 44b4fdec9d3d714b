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
