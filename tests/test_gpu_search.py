"""GPU parity of the triangulation search (Sec. 3): device flip walks against
the oracle's walk (same counter-based draws, bit-exact edge sets), programs
built on the device against the host builder word for word, every
(triangulation, witness) code against the oracle, the objectives against
the oracle's, and the annealing accept step against the oracle's rule."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from oracle import search as OS
from paper_2604_09221_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def pw():
    from paper_2604_09221_amd import patchwork

    assert torch.cuda.is_available()
    patchwork.lib()
    return patchwork


def edge_set(E):
    return {tuple(int(x) for x in e) for e in np.asarray(E).reshape(-1, 4)}


def canon_edges(E):
    return sorted(tuple(sorted([(int(a), int(b)), (int(c), int(e))])) for a, b, c, e in np.asarray(E).reshape(-1, 4))


@pytest.mark.parametrize("d,symmetric", [(4, False), (6, True), (8, False), (8, True), (9, True)])
def test_flip_walk_matches_oracle(pw, d, symmetric):
    from paper_2604_09221_amd import search as S

    start = I.standard_triangulation(d) if symmetric else I.lift_triangulation(d, 2, noise=1.0)
    n, steps, seed = 48, 40, 1234 + d
    print(f"flip walk d={d} symmetric={symmetric}", flush=True)
    adj = S.replicate(d, start, n)
    moves = torch.zeros(n, dtype=torch.int32, device="cuda")
    pw.flip_walk(d, adj, steps, symmetric, seed, step0=0, moves=moves)
    pw.flip_walk(d, adj, steps, symmetric, seed, step0=steps, moves=moves)   # resumable: a second call continues
    torch.cuda.synchronize()
    rows = adj.cpu().numpy()
    mv = moves.cpu().numpy()
    total_moves = 0
    for w in range(n):
        want_E, want_m = OS.flip_walk(d, start.tolist(), 2 * steps, symmetric, seed, w)
        got_E = pw.edges_from_adjacency(d, rows[w].view(np.uint64))
        assert canon_edges(got_E) == canon_edges(want_E), w
        assert mv[w] == want_m
        total_moves += want_m
        pw.Triangulation(d, got_E)                 # still a unimodular triangulation
        if symmetric:
            assert OS.is_symmetric(d, got_E)
    assert total_moves > n                         # the walks do move


@pytest.mark.parametrize("d", [3, 5, 7, 8, 9])
def test_device_programs_equal_host_programs(pw, d):
    from paper_2604_09221_amd import search as S

    n = 64
    adj = S.replicate(d, I.lift_triangulation(d, 1, noise=1.0), n)
    pw.flip_walk(d, adj, 50, False, 99)
    progs, bad = pw.build_programs(d, adj)
    torch.cuda.synchronize()
    assert not bad.cpu().numpy().any()
    P = progs.cpu().numpy().view(np.uint32)
    rows = adj.cpu().numpy()
    assert P.shape[1] == pw.program_words(d)
    for t in range(n):
        E = pw.edges_from_adjacency(d, rows[t].view(np.uint64))
        host = pw.Triangulation(d, E).program()
        assert np.array_equal(P[t], host), t


def test_bad_adjacency_is_flagged(pw):
    d = 5
    rows = pw.adjacency_from_edges(d, I.standard_triangulation(d))
    broken = rows.copy()
    broken[3] = 0                                  # point 3 loses every edge
    for q in range(64):
        broken[q] &= ~np.uint64(1 << 3)
    adj = torch.from_numpy(np.stack([rows, broken]).view(np.int64)).cuda()
    progs, bad = pw.build_programs(d, adj)
    torch.cuda.synchronize()
    b = bad.cpu().numpy()
    assert b[0] == 0 and b[1] != 0
    # the flagged program keeps no neighbour lists: evaluating it reads
    # only its own words and reports failures
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    codes = torch.zeros((2 * 64, 2), dtype=torch.int64, device="cuda")
    wm = np.zeros((64, 2), dtype=np.uint64)
    wm[:, 0] = I.random_masks(d, 3, 64)[:, 0]
    pw.scheme_programs(d, progs, torch.from_numpy(I.masks128(wm)).cuda(), codes=codes, err=err)
    torch.cuda.synchronize()
    got = codes.cpu().numpy().view(np.uint64)
    assert np.array_equal(got[:64], oracle.scheme_many(d, I.standard_triangulation(d), wm))
    assert int(err.item()) != 0


@pytest.mark.parametrize("d,n_tris,n_w", [(4, 17, 70), (6, 40, 129), (7, 25, 64), (8, 33, 100), (9, 9, 65)])
def test_scheme_programs_match_oracle(pw, d, n_tris, n_w):
    from paper_2604_09221_amd import search as S

    adj = S.replicate(d, I.standard_triangulation(d), n_tris)
    pw.flip_walk(d, adj, 30, d % 2 == 0, 7 * d)
    progs, bad = pw.build_programs(d, adj)
    wm = I.random_masks(d, 50 + d, n_w)
    wt = torch.from_numpy(I.masks128(wm)).cuda()
    codes = torch.zeros((n_tris * n_w, 2), dtype=torch.int64, device="cuda")
    h = pw.Histogram(4096)
    _, err = pw.scheme_programs(d, progs, wt, codes=codes, hist=h)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and not bad.cpu().numpy().any()
    got = codes.cpu().numpy().view(np.uint64).reshape(n_tris, n_w, 2)
    rows = adj.cpu().numpy()
    ref = {}
    for t in range(n_tris):
        E = pw.edges_from_adjacency(d, rows[t].view(np.uint64))
        want = oracle.scheme_many(d, E, wm, threads=THREADS)
        assert np.array_equal(got[t], want), t
        for w, (lo, hi) in enumerate(want):
            c = int(lo) | (int(hi) << 64)
            cnt, wi = ref.get(c, (0, t * n_w + w))
            ref[c] = (cnt + 1, min(wi, t * n_w + w))
    assert h.read() == ref


@pytest.mark.parametrize("mode", [0, 1])
def test_objective_matches_oracle(pw, mode):
    from paper_2604_09221_amd import search as S

    d, n_tris, n_w = 8, 20, 777
    adj = S.replicate(d, I.standard_triangulation(d), n_tris)
    pw.flip_walk(d, adj, 60, False, 5)
    progs, _ = pw.build_programs(d, adj)
    wm = I.random_masks(d, 8, n_w)
    codes = torch.zeros((n_tris * n_w, 2), dtype=torch.int64, device="cuda")
    pw.scheme_programs(d, progs, torch.from_numpy(I.masks128(wm)).cuda(), codes=codes)
    got_codes = codes.cpu().numpy().view(np.uint64).reshape(n_tris, n_w, 2)
    ints = [[int(lo) | (int(hi) << 64) for lo, hi in got_codes[t]] for t in range(n_tris)]
    # a target present in the sample
    target = OS.code_pn(ints[0][0])
    score = pw.tri_objective(d, codes, n_tris, n_w, mode, target)
    torch.cuda.synchronize()
    s = score.cpu().numpy()
    for t in range(n_tris):
        assert s[t] == OS.objective(ints[t], mode, target), t
    # code_pn against the oracle's depth reading of the same codes
    for c in ints[0][:50]:
        dep = oracle.oval_depths(c)
        assert OS.code_pn(c) == (sum(1 for x in dep if x % 2 == 1), sum(1 for x in dep if x % 2 == 0))


def test_anneal_accept_matches_oracle(pw):
    from paper_2604_09221_amd import search as S

    d, n = 6, 200
    cur = S.replicate(d, I.standard_triangulation(d), n)
    prop = cur.clone()
    pw.flip_walk(d, prop, 5, False, 77)
    best = cur.clone()
    rng = np.random.default_rng(4)
    sc = rng.integers(0, 40, n).astype(np.float32)
    sp = (sc + rng.integers(-6, 4, n)).astype(np.float32)
    sb = sc - 1
    score_cur = torch.from_numpy(sc.copy()).cuda()
    score_prop = torch.from_numpy(sp).cuda()
    score_best = torch.from_numpy(sb.copy()).cuda()
    table = S.accept_table(2.0)
    n_acc = torch.zeros(n, dtype=torch.int32, device="cuda")
    cur0, prop0 = cur.cpu().numpy(), prop.cpu().numpy()
    pw.anneal_accept(cur, prop, score_cur, score_prop, best, score_best,
                     torch.from_numpy(table.view(np.int32)).cuda(), 31, 9, n_acc)
    torch.cuda.synchronize()
    c1, p1, a1 = cur.cpu().numpy(), prop.cpu().numpy(), n_acc.cpu().numpy()
    s1, b1 = score_cur.cpu().numpy(), score_best.cpu().numpy()
    best1 = best.cpu().numpy()
    for w in range(n):
        take = OS.accept(float(sc[w]), float(sp[w]), [int(x) for x in table], 31, w, 9)
        want = prop0[w] if take else cur0[w]
        assert np.array_equal(c1[w], want) and np.array_equal(p1[w], want)
        assert a1[w] == int(take)
        assert s1[w] == (sp[w] if take else sc[w])
        assert b1[w] == max(sb[w], s1[w])
        if s1[w] > sb[w]:
            assert np.array_equal(best1[w], want)
    assert 0 < a1.sum() < n


def test_anneal_improves_and_keeps_valid_triangulations(pw):
    from paper_2604_09221_amd import search as S

    d = 6
    res = S.anneal(d, n_chains=64, iters=60, n_masks=512, mode=0, seed=3, log_every=20)
    assert (res.best_score >= res.final_score).all()
    rows = res.best.cpu().numpy()
    # the best scores are what the oracle computes on the same sample
    for t in range(0, 64, 16):
        E = pw.edges_from_adjacency(d, rows[t].view(np.uint64))
        pw.Triangulation(d, E)
        codes = oracle.scheme_many(d, E, res.masks, threads=THREADS)
        assert OS.objective([int(lo) | (int(hi) << 64) for lo, hi in codes], 0) == res.best_score[t]
    start = OS.objective([int(lo) | (int(hi) << 64) for lo, hi in
                          oracle.scheme_many(d, I.standard_triangulation(d), res.masks, threads=THREADS)], 0)
    assert res.best_score.max() > start


def test_objective_novelty_mode(pw):
    """mode 2 counts the distinct codes outside a known list."""
    from paper_2604_09221_amd import search as S

    d, n_tris, n_w = 7, 12, 500
    adj = S.replicate(d, I.standard_triangulation(d), n_tris)
    pw.flip_walk(d, adj, 40, False, 11)
    progs, _ = pw.build_programs(d, adj)
    wm = I.random_masks(d, 12, n_w)
    codes = torch.zeros((n_tris * n_w, 2), dtype=torch.int64, device="cuda")
    pw.scheme_programs(d, progs, torch.from_numpy(I.masks128(wm)).cuda(), codes=codes)
    c = codes.cpu().numpy().view(np.uint64).reshape(n_tris, n_w, 2)
    ints = [[int(lo) | (int(hi) << 64) for lo, hi in c[t]] for t in range(n_tris)]
    known = sorted(set(ints[0]))[::2]
    score = pw.tri_objective(d, codes, n_tris, n_w, 2, known=S.known_tensor(known))
    torch.cuda.synchronize()
    s = score.cpu().numpy()
    for t in range(n_tris):
        assert s[t] == len(set(ints[t]) - set(known)), t


@pytest.mark.parametrize("d,want", [
    (4, {6, 26, 106, 426, 28}),                                  # <1> <2> <3> <4> <1<1>>
    (5, None),                                                   # <J + k>, k <= 6, and <J + 1<1>>
])
def test_iterate_realises_the_small_degree_classification(pw, d, want):
    """The witness <-> triangulation loop from the standard triangulation
    finds every non-empty real scheme of degree 4 and 5 (Sec. 3: for d <= 5
    all of them are T-curves) and nothing else, each with a regular
    triangulation and a witness the oracle confirms."""
    from paper_2604_09221_amd import search as S

    if want is None:
        J = oracle.J_BIT
        want = {oracle.code_from_forest([[]] * k, True) for k in range(0, 7)} | {28 | J}
    res = S.iterate(d, [I.standard_triangulation(d)], n_tris=512, walk_steps=16, max_rounds=4, seed=2,
                    explore_chains=64, explore_iters=30, explore_masks=256)
    assert set(res.found) == want
    for code, r in res.found.items():
        assert oracle.scheme(d, r.edges, r.mask) == code


def degree6_schemes():
    """The non-empty real schemes of degree 6, from the constraints that
    decide them: Bezout (depth <= 3; a nest of depth 3 has no other oval;
    no two non-empty nests), Harnack (at most 11 ovals), Gudkov-Rokhlin for
    M-curves (p - n = 1 mod 8) and Gudkov-Krakhnov-Kharlamov for
    (M-1)-curves (p - n = 0 or 2 mod 8); every scheme these allow is
    realised (Gudkov's classification; the paper counts 55)."""
    out = {oracle.code_from_forest([[[[]]]], False)}                     # <1<1<1>>>
    for a in range(1, 11):                                                # <a>
        p, n = a, 0
        if a == 10 and (p - n) % 8 not in (0, 2):
            continue
        out.add(oracle.code_from_forest([[]] * a, False))
    for b in range(1, 11):                                                # <1<b> + a>
        for a in range(0, 11 - b):
            p, n = a + 1, b
            total = a + 1 + b
            if total == 11 and (p - n) % 8 != 1:
                continue
            if total == 10 and (p - n) % 8 not in (0, 2):
                continue
            out.add(oracle.code_from_forest([[[]] * b] + [[]] * a, False))
    return out


def test_search_realises_all_55_degree6_schemes(pw):
    """Annealing over triangulations, then the witness <-> triangulation loop
    (Sec. 3): every non-empty real scheme of degree six, each with a regular
    triangulation (exact certificate) and a witness the oracle confirms."""
    from paper_2604_09221_amd import regular
    from paper_2604_09221_amd import search as S

    want = degree6_schemes()
    assert len(want) == 55
    d = 6
    ann = S.anneal(d, n_chains=256, iters=300, n_masks=1024, mode=0, seed=1)
    rows = ann.best.cpu().numpy()
    pool, keys = [I.standard_triangulation(d)], set()
    for t in np.argsort(-ann.best_score):
        E = pw.edges_from_adjacency(d, rows[t].view(np.uint64))
        k = pw.canonical(d, E)[0].tobytes()
        if k not in keys and regular.is_regular(d, E):
            keys.add(k)
            pool.append(E)
        if len(pool) > 8:
            break
    res = S.iterate(d, pool, n_tris=4096, walk_steps=64, max_rounds=10, seed=1, target_count=55)
    assert set(res.found) == want
    for code, r in res.found.items():
        assert regular.certificate(d, r.edges) is not None
        assert oracle.scheme(d, r.edges, r.mask) == code
