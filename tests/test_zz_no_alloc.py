"""patchwork_scheme_batch_multi_noalloc (the allocation-free variant of the
batched multi-triangulation call, for callers that cannot allocate device
memory) against patchwork_scheme_batch_multi: the same codes and the same
histograms, on two calls in a row, the second with a smaller input, and the
size limits rejected before anything is launched."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2604_09221_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pw():
    from paper_2604_09221_amd import patchwork

    assert torch.cuda.is_available()
    patchwork.lib()
    return patchwork


def workload(n_tris, per_tri, seed):
    degs = I.batched_degrees(n_tris, seed)
    edges = [I.lift_triangulation(int(d), t, noise=1.0) for t, d in enumerate(degs)]
    counts = [per_tri + (t * 13) % 97 for t in range(n_tris)]     # ragged
    masks = [I.random_masks(int(d), 500 + t, c) for t, (d, c) in enumerate(zip(degs, counts))]
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return degs, edges, np.vstack(masks), offsets


def run_both(pw, tris, masks, offsets, config):
    mt = torch.from_numpy(I.masks128(masks)).cuda()
    out = []
    for noalloc in (False, True):
        codes = torch.zeros((len(masks), 2), dtype=torch.int64, device="cuda")
        hists = [pw.Histogram(2048) for _ in tris]
        pw.batch_multi(tris, mt, offsets, hists=hists, codes=codes, config=config, noalloc=noalloc)
        torch.cuda.synchronize()
        out.append((codes.cpu().numpy(), [h.read() for h in hists]))
    return out


def test_noalloc_matches_batch_multi_two_calls(pw):
    print("noalloc: call 1 (36 triangulations, d 4..12, ~3000 masks each)", flush=True)
    degs, edges, masks, offsets = workload(36, 3000, seed=21)
    assert {4, 12} <= {int(d) for d in degs}
    tris = [pw.Triangulation(int(d), E) for d, E in zip(degs, edges)]
    (c_ref, h_ref), (c_na, h_na) = run_both(pw, tris, masks, offsets, (512, 1, 0))
    assert np.array_equal(c_ref, c_na)
    assert (c_na != 0).any(axis=1).all()
    assert h_ref == h_na
    for t in tris:
        assert t.errors() == 0
    print("noalloc: call 2 (smaller: 7 triangulations, ~700 masks each)", flush=True)
    degs2, edges2, masks2, offsets2 = workload(7, 700, seed=22)
    tris2 = [pw.Triangulation(int(d), E) for d, E in zip(degs2, edges2)]
    (c_ref2, h_ref2), (c_na2, h_na2) = run_both(pw, tris2, masks2, offsets2, (256, 2, 0))
    assert np.array_equal(c_ref2, c_na2)
    assert h_ref2 == h_na2
    # every mask's count appears once: the histograms sum to the call's size
    assert sum(c for h in h_na2 for c, _ in h.values()) == len(masks2)


def test_noalloc_limits(pw):
    degs, edges, masks, offsets = workload(2, 64, seed=23)
    tris = [pw.Triangulation(int(d), E) for d, E in zip(degs, edges)]
    # a mask buffer as large as the offsets below name (zeros), so that the
    # call would stay in bounds even if it were not refused
    n_big = 64 * 300000 + 1
    mt = torch.zeros(2 * n_big, dtype=torch.int64, device="cuda")
    codes = torch.zeros((n_big, 2), dtype=torch.int64, device="cuda")
    # more work items than the fixed table holds: refused, nothing written
    big = np.array([0, n_big - 1, n_big], dtype=np.int64)
    with pytest.raises(pw.PatchworkError) as e:
        pw.batch_multi(tris, mt, big, codes=codes, config=(64, 1, 0), noalloc=True)
    assert e.value.status == pw.PW_ERR_ARG
    # more triangulations than the descriptor table holds
    many = tris * 2049
    off = np.zeros(len(many) + 1, dtype=np.int64)
    with pytest.raises(pw.PatchworkError) as e:
        pw.batch_multi(many, mt, off, codes=codes, config=(64, 1, 0), noalloc=True)
    assert e.value.status == pw.PW_ERR_ARG
    torch.cuda.synchronize()
    assert not codes.cpu().numpy().any()
