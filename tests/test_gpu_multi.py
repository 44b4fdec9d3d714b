"""GPU parity of the batched multi-triangulation call
(patchwork_scheme_batch_multi): uneven degrees 4..12 in one call, codes
bit-exact against the oracle, per-triangulation histograms equal to the
codes' histograms, and identical tables under different launch shapes,
including every lane-group size (1, 2 or 4 lanes per mask) for degrees
8..12."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
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


def workload(n_tris, per_tri, seed, noise=1.0):
    degs = I.batched_degrees(n_tris, seed)
    edges = [I.lift_triangulation(int(d), t, noise=noise) for t, d in enumerate(degs)]
    counts = [per_tri + (t * 7) % 61 for t in range(n_tris)]     # ragged
    masks = [I.random_masks(int(d), 1000 + t, c) for t, (d, c) in enumerate(zip(degs, counts))]
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return degs, edges, masks, offsets


def hist_of(codes2, base):
    keys, inv, counts = np.unique(codes2, axis=0, return_inverse=True, return_counts=True)
    wmin = np.full(len(keys), np.iinfo(np.uint64).max, dtype=np.uint64)
    np.minimum.at(wmin, inv.reshape(-1), np.arange(base, base + len(codes2), dtype=np.uint64))
    return {int(lo) | (int(hi) << 64): (int(c), int(w)) for (lo, hi), c, w in zip(keys, counts, wmin)}


def test_multi_codes_and_histograms(pw):
    degs, edges, masks, offsets = workload(27, 2048, seed=5)
    tris = [pw.Triangulation(int(d), E) for d, E in zip(degs, edges)]
    allm = np.vstack(masks)
    mt = torch.from_numpy(I.masks128(allm)).cuda()
    codes = torch.empty((len(allm), 2), dtype=torch.int64, device="cuda")
    hists = [pw.Histogram(1024) for _ in tris]
    pw.batch_multi(tris, mt, offsets, hists=hists, codes=codes, config=(1024, 1, 0))
    got = codes.cpu().numpy().view(np.uint64)
    for t, (d, E) in enumerate(zip(degs, edges)):
        a, b = offsets[t], offsets[t + 1]
        want = oracle.scheme_many(int(d), E, masks[t], threads=THREADS)
        assert np.array_equal(got[a:b], want), (t, int(d))
        assert hists[t].read() == hist_of(want, a), (t, int(d))
        assert tris[t].errors() == 0
    # another launch shape, one lane per mask everywhere: the same tables
    hists2 = [pw.Histogram(1024) for _ in tris]
    pw.batch_multi(tris, mt, offsets, hists=hists2, config=(4096, 2, 2, 0))
    for h1, h2 in zip(hists, hists2):
        assert h1.read() == h2.read()
    # four waves per block: each LDS class lowers it until its block fits
    # (3 at d = 12, 4 at d = 11 and below)
    assert {10, 11, 12} <= {int(d) for d in degs}
    # (and two lanes per mask for degrees 8..12)
    hists3 = [pw.Histogram(1024) for _ in tris]
    codes3 = torch.zeros_like(codes)
    g2 = pw.lane_groups_code({d: 2 for d in range(8, 13)})
    pw.batch_multi(tris, mt, offsets, hists=hists3, codes=codes3, config=(512, 4, 0, g2))
    assert torch.equal(codes3, codes)
    for h1, h3 in zip(hists, hists3):
        assert h1.read() == h3.read()


def test_multi_literal_lift_slots_and_edge_cases(pw):
    """Literal lifts (noise 0.05) give the standard triangulation for every
    seed; every slot must still be evaluated from its own handle."""
    degs, edges, masks, offsets = workload(18, 512, seed=9, noise=0.05)
    tris = [pw.Triangulation(int(d), E) for d, E in zip(degs, edges)]
    allm = np.vstack(masks)
    mt = torch.from_numpy(I.masks128(allm)).cuda()
    codes = torch.empty((len(allm), 2), dtype=torch.int64, device="cuda")
    pw.batch_multi(tris, mt, offsets, codes=codes)
    got = codes.cpu().numpy().view(np.uint64)
    pick = np.random.default_rng(0).choice(len(allm), 512, replace=False)
    for k in pick:
        t = int(np.searchsorted(offsets, k, side="right") - 1)
        want = oracle.scheme_many(int(degs[t]), edges[t], allm[k:k + 1])
        assert np.array_equal(got[k:k + 1], want)
    # empty slots are allowed ...
    off2 = offsets.copy()
    off2[3] = off2[2]
    off2[4] = off2[2]
    codes2 = torch.zeros_like(codes)
    pw.batch_multi(tris, mt, off2, codes=codes2)                 # slot 4 now owns [off2[4], off2[5])
    got2 = codes2.cpu().numpy().view(np.uint64)
    a, b = int(off2[4]), int(off2[5])
    assert np.array_equal(got2[a:b], oracle.scheme_many(int(degs[4]), edges[4], allm[a:b], threads=8))
    assert np.array_equal(got2[b:], got[b:])
    assert np.array_equal(got2[:a], got[:a])
    # a call in which only slot 5 has masks: the launches of the other
    # degrees' LDS classes have no items and are skipped
    off4 = offsets.copy()
    off4[:6] = offsets[5]
    off4[6:] = offsets[6]
    assert len({int(d) for d in degs}) > 1
    codes4 = torch.zeros_like(codes)
    pw.batch_multi(tris, mt, off4, codes=codes4)
    got4 = codes4.cpu().numpy().view(np.uint64)
    a, b = int(offsets[5]), int(offsets[6])
    assert np.array_equal(got4[a:b], got[a:b])
    assert not got4[:a].any() and not got4[b:].any()
    # ... decreasing offsets are not
    off3 = offsets.copy()
    off3[3] = off3[2] - 1
    with pytest.raises(pw.PatchworkError):
        pw.batch_multi(tris, mt, off3, codes=codes)
    empty = np.zeros(len(tris) + 1, dtype=np.int64)
    pw.batch_multi(tris, mt, empty, codes=codes)                 # nothing to do


@pytest.mark.parametrize("groups", [{}, {10: 4, 11: 4, 12: 4, 9: 2}, {10: 2, 11: 2, 12: 2}])
def test_multi_many_regions_take_the_overflow_path(pw, groups):
    """Degrees 10..12 run with phase-4 tables for at most 32 regions; masks
    with more (Harnack: 38, 46, 57 regions, and near-Harnack masks) are
    evaluated again with the full tables.  Codes, histograms (counts and
    witnesses) and error flags must be as for any other mask, with one lane
    per mask and with lane groups."""
    rng = np.random.default_rng(9)
    degs = [10, 11, 12, 9, 12]
    edges = [I.standard_triangulation(d) if k % 2 == 0 else I.lift_triangulation(d, 40 + k, noise=1.0)
             for k, d in enumerate(degs)]
    masks = []
    for k, d in enumerate(degs):
        nA = I.n_points(d)
        h = I.harnack_mask(d)
        rows = [h] + [h ^ (1 << int(b)) for b in rng.integers(1, nA, size=150)]
        rows += [h ^ (1 << int(a)) ^ (1 << int(b)) for a, b in rng.integers(1, nA, size=(100, 2))]
        m = np.zeros((len(rows) + 300, 2), dtype=np.uint64)
        m[:len(rows), 0] = [x & ((1 << 64) - 1) for x in rows]
        m[:len(rows), 1] = [x >> 64 for x in rows]
        m[len(rows):] = I.random_masks(d, 77 + k, 300)
        masks.append(m)
    offsets = np.concatenate([[0], np.cumsum([len(m) for m in masks])]).astype(np.int64)
    tris = [pw.Triangulation(int(d), E) for d, E in zip(degs, edges)]
    allm = np.vstack(masks)
    mt = torch.from_numpy(I.masks128(allm)).cuda()
    codes = torch.empty((len(allm), 2), dtype=torch.int64, device="cuda")
    hists = [pw.Histogram(4096) for _ in tris]
    pw.batch_multi(tris, mt, offsets, hists=hists, codes=codes, config=(256, 1, 0, pw.lane_groups_code(groups)))
    got = codes.cpu().numpy().view(np.uint64)
    many = 0
    for t, (d, E) in enumerate(zip(degs, edges)):
        a, b = offsets[t], offsets[t + 1]
        want = oracle.scheme_many(int(d), E, masks[t], threads=THREADS)
        assert np.array_equal(got[a:b], want), (t, int(d))
        assert hists[t].read() == hist_of(want, a), (t, int(d))
        assert tris[t].errors() == 0
        if d >= 10:
            many += sum(oracle.n_ovals(int(lo) | (int(hi) << 64)) + 1 > 32 for lo, hi in want)
    assert many > 100   # the overflow path did run


@pytest.mark.parametrize("G,wpb,chunk", [(2, 1, 256), (4, 1, 256), (4, 4, 1000), (2, 2, 333)])
def test_multi_lane_groups_every_degree(pw, G, wpb, chunk):
    """G lanes per mask for every degree 8..12: codes equal the oracle's for
    every mask (standard and lifted triangulations, the Harnack mask and its
    single flips, all '+', random masks; per-triangulation counts that are
    not multiples of the 64 / G masks a wave holds), histograms equal the
    codes' histograms and those of the one-lane call, and no error flags."""
    degs = [8, 9, 10, 11, 12, 8, 10, 12]
    edges = [I.standard_triangulation(d) if k < 5 and k % 2 == 0 else I.lift_triangulation(d, 60 + k, noise=1.0)
             for k, d in enumerate(degs)]
    masks = []
    for k, d in enumerate(degs):
        nA = I.n_points(d)
        h = I.harnack_mask(d)
        rows = [h, 0] + [h ^ (1 << b) for b in range(1, nA, 2)]
        m = np.zeros((len(rows) + 700 + 13 * k, 2), dtype=np.uint64)
        m[:len(rows), 0] = [x & ((1 << 64) - 1) for x in rows]
        m[:len(rows), 1] = [x >> 64 for x in rows]
        m[len(rows):] = I.random_masks(d, 300 + k, len(m) - len(rows))
        masks.append(m)
    offsets = np.concatenate([[0], np.cumsum([len(m) for m in masks])]).astype(np.int64)
    tris = [pw.Triangulation(int(d), E) for d, E in zip(degs, edges)]
    allm = np.vstack(masks)
    mt = torch.from_numpy(I.masks128(allm)).cuda()
    code = pw.lane_groups_code({d: G for d in range(8, 13)})
    codes = torch.zeros((len(allm), 2), dtype=torch.int64, device="cuda")
    hists = [pw.Histogram(4096) for _ in tris]
    pw.batch_multi(tris, mt, offsets, hists=hists, codes=codes, config=(chunk, wpb, 0, code))
    got = codes.cpu().numpy().view(np.uint64)
    for t, (d, E) in enumerate(zip(degs, edges)):
        a, b = offsets[t], offsets[t + 1]
        want = oracle.scheme_many(int(d), E, masks[t], threads=THREADS)
        assert np.array_equal(got[a:b], want), (t, int(d))
        assert hists[t].read() == hist_of(want, a), (t, int(d))
        assert tris[t].errors() == 0
    # mixed: one, two and four lanes per mask in one call
    mixed = pw.lane_groups_code({8: 1, 9: 4, 10: 2, 11: 1, 12: G})
    hists1 = [pw.Histogram(4096) for _ in tris]
    pw.batch_multi(tris, mt, offsets, hists=hists1, config=(chunk, wpb, 0, mixed))
    for h, h1 in zip(hists, hists1):
        assert h.read() == h1.read()


def test_multi_lane_groups_refused_below_degree_8(pw):
    tris = [pw.Triangulation(7, I.standard_triangulation(7))]
    mt = torch.zeros((64, 2), dtype=torch.int64, device="cuda")
    codes = torch.zeros((64, 2), dtype=torch.int64, device="cuda")
    for groups in ({7: 2}, {7: 4}):
        with pytest.raises(pw.PatchworkError):
            pw.batch_multi(tris, mt.view(-1), [0, 64], codes=codes, config=(256, 1, 0, pw.lane_groups_code(groups)))
    with pytest.raises(pw.PatchworkError):
        pw.batch_multi(tris, mt.view(-1), [0, 64], codes=codes, config=(256, 1, 0, 3 << 20))


def test_multi_full_size_sampled(pw):
    """The batched workload at full size, in the launch shape the benchmark
    uses (the tuned shape for this degree mix): 4096 triangulations of
    degrees 4..12 (literal lifts, seeds 0..4095), 2^16 generated masks each,
    codes and per-triangulation histograms in one call.  Three masks per
    triangulation (first, last, one inside) are checked against the oracle;
    on a sample of triangulations the histogram counts every mask, holds each
    sampled code, and names a witness no later than the sampled mask."""
    import bench
    from paper_2604_09221_amd import learn as Lr

    n_tris, per = 4096, 1 << 16
    degs = I.batched_degrees(n_tris, 0)
    edges = [I.lift_triangulation(int(d), t, noise=0.05) for t, d in enumerate(degs)]
    tris = [pw.Triangulation(int(d), E) for d, E in zip(degs, edges)]
    masks = torch.empty((n_tris * per, 2), dtype=torch.int64, device="cuda")
    for t, d in enumerate(degs):
        masks[t * per:(t + 1) * per] = Lr.random_masks(t, 0, per, I.n_points(int(d)))
    offsets = np.arange(n_tris + 1, dtype=np.int64) * per
    hists = [pw.Histogram(bench.hist_capacity(int(d))) for d in degs]
    codes = torch.zeros((n_tris * per, 2), dtype=torch.int64, device="cuda")
    pw.batch_multi(tris, masks.view(-1), offsets, hists=hists, codes=codes)
    rng = np.random.default_rng(5)
    inner = rng.integers(1, per - 1, size=n_tris)
    idx = np.stack([offsets[:-1], offsets[:-1] + inner, offsets[1:] - 1], axis=1)
    sel = torch.from_numpy(idx.reshape(-1)).cuda()
    got = codes[sel].cpu().numpy().view(np.uint64).reshape(n_tris, 3, 2)
    m = masks[sel].cpu().numpy().view(np.uint64).reshape(n_tris, 3, 2)
    for t, d in enumerate(degs):
        want = oracle.scheme_many(int(d), edges[t], m[t])
        assert np.array_equal(got[t], want), (t, int(d))
        assert tris[t].errors() == 0
    for t in rng.choice(n_tris, 48, replace=False):
        h = hists[t].read()
        assert sum(c for c, _ in h.values()) == per, t
        for j in range(3):
            code = int(got[t, j, 0]) | (int(got[t, j, 1]) << 64)
            assert code in h and h[code][1] <= idx[t, j], (t, j)
