"""What the trained network adds to the proposal search.

The network is trained on the GPU (project kernels) on masks labelled by the
exact kernel.  Mutants of the rarest schemes' witnesses are then ranked by
the network; every mutant is also judged by the exact kernel.  The true
feature rarity of the network's top 10% must beat that of a random 10% --
the ranking the ablation uses -- and so must their share of schemes never
seen in the training set."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2604_09221_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_network_ranking_beats_random_ranking():
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
    labels = lab.cpu().numpy()
    st = np.concatenate([[0], np.cumsum(Lr.HEADS)])
    rar = np.zeros(Lr.OUT, dtype=np.float32)
    for h in range(6):
        p = np.bincount(labels[:, h], minlength=Lr.HEADS[h]).astype(np.float64) + 0.5
        rar[st[h]:st[h + 1]] = -np.log(p / p.sum())
    hist = pw.Histogram(1 << 12)
    tri.histogram(m[:, 0].contiguous(), hist)
    seen = set(hist.read())
    parents, _ = Lr.rarest_witnesses(hist, m, 2048)
    cand = Lr.mutate(parents, 1 << 16, nA, 2, 12345)
    sc = Lr.score(net.forward(Lr.encode(cand, cand.shape[0], nA)), torch.from_numpy(rar).cuda()).cpu().numpy()
    true_codes = tri.batch(cand[:, 0].contiguous())
    tl = Lr.features(true_codes).cpu().numpy()
    true_rarity = sum(rar[st[h] + tl[:, h]] for h in range(6))
    c = true_codes.cpu().numpy().view(np.uint64)
    novel = np.array([(int(a) | (int(b) << 64)) not in seen for a, b in c])
    k = len(sc) // 10
    top = np.argsort(-sc)[:k]
    rnd = np.random.default_rng(0).choice(len(sc), k, replace=False)
    assert true_rarity[top].mean() > 1.1 * true_rarity[rnd].mean()
    assert novel[top].mean() >= novel[rnd].mean()
    assert tri.errors() == 0
