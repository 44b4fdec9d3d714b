"""The fact behind the even-degree sweep kernel's per-chunk merge, checked on
its own, in plain Python, independently of the kernels and of the oracle.

In a chunk of the sweep kernel only the lattice points with bits 1..9
(point order of inputs.points: j-major) change sign; the other points'
diamond vertices have fixed signs.  The kernel merges into its snapshot, with
no odd-cycle flag, every set of the pair graph (sets of same-sign connected
fixed vertices, joined by the antipodal pairs of fixed boundary vertices)
that no varying vertex reaches.  That is right only if such a set never
holds a cycle closed by an odd number of pairs (a one-sided loop of RP^2).
The reason given: bits 1..d are the points (i, 0), so the varying vertices
cover the horizontal axis of the reflected diamond except its centre, a
one-sided loop that every other one-sided loop crosses; so an odd cycle of
fixed vertices passes through the centre (0, 0), whose neighbours vary.

Here the reflected diamond (eq. (signs) of Sec. 2: the copy in quadrant
(ex, ey) takes sigma(|x|, |y|) flipped by |x| if x < 0 and by |y| if
y < 0), its same-sign components and the antipodal identification of
Sec. 2 are built from the edge list, and the claim is tested on random
fixed-sign patterns of the Fig. 2 triangulations and of standard and
varied ones at d = 6 and 8 -- together with checks that the situations it
is about do occur (sets out of reach, odd cycles within reach)."""
from __future__ import annotations

import os

import numpy as np
import pytest

from paper_2604_09221_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def _diamond(d, edges):
    """Vertices (x, y) with |x| + |y| <= d, the reflected edges, and the
    antipodal pairs {p, -p} of boundary vertices (deduplicated)."""
    verts = [(x, y) for y in range(-d, d + 1) for x in range(-d, d + 1) if abs(x) + abs(y) <= d]
    index = {p: k for k, p in enumerate(verts)}
    es = set()
    for i0, j0, i1, j1 in np.asarray(edges).reshape(-1, 4).tolist():
        for ex in (1, -1):
            for ey in (1, -1):
                a, b = index[(ex * i0, ey * j0)], index[(ex * i1, ey * j1)]
                es.add((min(a, b), max(a, b)))
    pairs = set()
    for (x, y) in verts:
        if abs(x) + abs(y) == d:
            a, b = index[(x, y)], index[(-x, -y)]
            pairs.add((min(a, b), max(a, b)))
    return verts, sorted(es), sorted(pairs)


def _find(par, x):
    while par[x] != x:
        par[x] = par[par[x]]
        x = par[x]
    return x


def _claim_counts(d, edges, n_patterns, seed, varying_bits=range(1, 10)):
    verts, es, pairs = _diamond(d, edges)
    pts = I.points(d)
    bit_of = {p: k for k, p in enumerate(pts)}
    lat = [bit_of[(abs(x), abs(y))] for (x, y) in verts]
    varying_bits = set(varying_bits)
    vary = [b in varying_bits for b in lat]
    nbr = [[] for _ in verts]
    for a, b in es:
        nbr[a].append(b)
        nbr[b].append(a)
    rng = np.random.default_rng(seed)
    untouched_sets = odd_reached = violations = 0
    for _ in range(n_patterns):
        sigma = rng.integers(0, 2, len(pts))
        sigma[0] = 0
        sign = [(int(sigma[lat[k]]) + (abs(x) if x < 0 else 0) + (abs(y) if y < 0 else 0)) % 2
                for k, (x, y) in enumerate(verts)]
        # same-sign components of the fixed part (the snapshot's sets)
        par = list(range(len(verts)))
        for a, b in es:
            if not vary[a] and not vary[b] and sign[a] == sign[b]:
                ra, rb = _find(par, a), _find(par, b)
                if ra != rb:
                    par[max(ra, rb)] = min(ra, rb)
        # sets reached by a varying vertex: a fixed vertex with a varying
        # neighbour, or a fixed end of a pair whose other end varies
        reached = set()
        for v in range(len(verts)):
            if not vary[v] and any(vary[u] for u in nbr[v]):
                reached.add(_find(par, v))
        for a, b in pairs:
            if vary[a] != vary[b]:
                reached.add(_find(par, b if vary[a] else a))
        # the pair graph over the sets, with parity 1 per pair
        kp = {}
        kpar = {}
        odd = {}

        def kfind(x):
            p = 0
            while kp.get(x, x) != x:
                p ^= kpar[x]
                x = kp[x]
            return x, p

        for a, b in pairs:
            if vary[a] or vary[b]:
                continue
            (ra, pa), (rb, pb) = kfind(_find(par, a)), kfind(_find(par, b))
            if ra == rb:
                if pa == pb:
                    odd[ra] = True
            else:
                lo, hi = min(ra, rb), max(ra, rb)
                kp[hi], kpar[hi] = lo, pa ^ pb ^ 1
                odd[lo] = odd.get(lo, False) or odd.get(hi, False)
        # per component of the pair graph: reached, odd
        comp_reached = {}
        sets = {_find(par, v) for v in range(len(verts)) if not vary[v]}
        for s in sets:
            r, _ = kfind(s)
            comp_reached[r] = comp_reached.get(r, False) or (s in reached)
        for r, is_reached in comp_reached.items():
            if not is_reached:
                untouched_sets += 1
                if odd.get(r, False):
                    violations += 1
            elif odd.get(r, False):
                odd_reached += 1
    return untouched_sets, odd_reached, violations


def _fig2(name):
    return np.loadtxt(os.path.join(HERE, "golden", f"fig2_{name}.edges"), dtype=np.int32)


@pytest.mark.parametrize("d,which", [(8, "bow_tie"), (8, "rank016"), (8, "rank015"), (8, "standard"),
                                     (6, "standard"), (6, "varied")])
def test_unreached_pair_sets_have_no_odd_cycle(d, which):
    if which == "standard":
        edges = I.standard_triangulation(d)
    elif which == "varied":
        edges = I.lift_triangulation(d, 3, noise=1.0)
    else:
        edges = _fig2(which)
    untouched, odd_reached, violations = _claim_counts(d, edges, 300, seed=d)
    assert violations == 0
    assert untouched > 0          # the merge has something to do
    if which == "bow_tie":
        assert odd_reached > 0    # odd cycles occur, within reach (marks left to the batches)


@pytest.mark.parametrize("d", [6, 8])
def test_detector_finds_the_one_sided_region_when_nothing_varies(d):
    """Control: with no varying point every set is out of reach, and each
    sign distribution of even degree has exactly one region with an odd
    cycle (the non-orientable one, Sec. 2) -- so the check above would see
    one violation per pattern if the varying points did not cover the
    axis."""
    n = 100
    untouched, odd_reached, violations = _claim_counts(d, I.standard_triangulation(d), n, seed=1, varying_bits=())
    assert odd_reached == 0 and violations == n
