"""Host checks of the search-space symmetries (Sec. 3, Table 1): the S3
canonical form of triangulations, the point permutations and the (Z/2)^3
class representatives.  No GPU: these are host calls of the library.

Pins: the orbit counts of Table 1 (2 orbits at d=2, both symmetric; 18 at
d=3, 7 symmetric; at d=4, 74 symmetric orbits and 1278 regular ones, which
with the single non-regular orbit found by the regularity check make 1279
orbits of flip-connected unimodular triangulations), the S3 action written
out independently in tests/checkers.py, and the oracle's codes."""
from __future__ import annotations

import random

import numpy as np
import pytest

import checkers as K
import oracle
from paper_2604_09221_amd import inputs as I
from paper_2604_09221_amd import orbits
from paper_2604_09221_amd import patchwork as pw


def orbit_table(d):
    Ts = K.all_triangulations(d, I.standard_triangulation(d).tolist())
    orbs = {}
    for T in Ts:
        c, _, st = pw.canonical(d, T)
        orbs.setdefault(c.tobytes(), (st, T))
    return Ts, orbs


@pytest.mark.parametrize("d,n_orbits,n_sym", [(2, 2, 2), (3, 18, 7)])
def test_orbit_counts_table1_small(d, n_orbits, n_sym):
    _, orbs = orbit_table(d)
    assert len(orbs) == n_orbits
    # symmetric: some member is fixed by (x, y) -> (y, x), i.e. the
    # stabiliser contains a transposition (order 2 or 6, not 3)
    assert sum(st in (2, 6) for st, _ in orbs.values()) == n_sym


def test_orbit_counts_d4():
    Ts, orbs = orbit_table(4)
    assert len(Ts) == 7424
    assert sum(st in (2, 6) for st, _ in orbs.values()) == 74           # Table 1
    assert len(orbs) == 1279                                              # 1278 regular + 1 (regularity tests)
    # orbit-stabiliser: the orbit sizes add up to the number of triangulations
    assert sum(6 // st for st, _ in orbs.values()) == len(Ts)


def _edge_key(d, E):
    return sorted(tuple(sorted([(a, b), (c, e)], key=lambda p: I.points(d).index(p))) for (a, b, c, e) in E)


@pytest.mark.parametrize("d", [5, 6, 7, 8, 9])
def test_canonical_is_an_orbit_invariant(d):
    for seed in range(3):
        E = [tuple(int(x) for x in e) for e in I.lift_triangulation(d, seed, noise=1.0)]
        c0, k0, st0 = pw.canonical(d, E)
        images = []
        for f in K.s3_maps(d):
            E2, _ = K.act_s3(d, E, 0, f)
            c, k, st = pw.canonical(d, E2)
            assert np.array_equal(c, c0) and st == st0
            images.append(tuple(map(tuple, _edge_key(d, E2))))
        assert len(set(images)) * st0 == 6
        # the returned permutation maps the input to the canonical member
        E3, _ = K.act_s3(d, E, 0, K.s3_maps(d)[k0])
        assert _edge_key(d, E3) == _edge_key(d, [tuple(x) for x in c0.tolist()])


def test_stabilizers_of_known_triangulations():
    for d in range(1, 13):
        assert pw.canonical(d, I.standard_triangulation(d))[2] == 6
    from test_oracle_pins import fig2

    E, _ = fig2("rank016")
    assert pw.canonical(8, E)[2] in (2, 6)          # fixed by x <-> y


@pytest.mark.parametrize("d", [1, 3, 6, 12])
def test_point_map_is_the_s3_action(d):
    pts = I.points(d)
    for k, f in enumerate(K.s3_maps(d)):
        pm = pw.point_map(d, k)
        assert sorted(pm.tolist()) == list(range(len(pts)))
        for p, q in enumerate(pm):
            assert pts[int(q)] == f(pts[p])


@pytest.mark.parametrize("d", range(2, 13))
def test_class_fixed_bits(d):
    fz = pw.class_fixed_bits(d)
    pts = I.points(d)
    ks = [k for k in range(len(pts)) if (fz >> k) & 1]
    assert len(ks) == 3 and ks[0] == 0
    assert len({(pts[k][0] % 2, pts[k][1] % 2) for k in ks}) == 3
    if d >= 4:
        assert all(k >= 10 for k in ks[1:])          # lattice points 1..9 stay free


def test_class_representatives_cover_every_mask_once():
    d = 4
    fz = pw.class_fixed_bits(d)
    free = ((1 << I.n_points(d)) - 1) & ~fz
    seen = np.zeros(1 << I.n_points(d), dtype=np.int32)
    for idx in range(1 << (I.n_points(d) - 3)):
        m = I.pdep(idx, free)
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    seen[K.affine_flip(d, m, a, b, c)] += 1
    assert (seen == 1).all()


def test_orbit_witness_maps_back_to_the_input():
    rng = random.Random(5)
    for d, seed in ((5, 0), (6, 1), (7, 0)):
        E = I.lift_triangulation(d, seed, noise=1.0)
        canon, k, st = pw.canonical(d, E)
        res = orbits.OrbitSweep(d, canon, k, st, pw.class_fixed_bits(d), 1 << (I.n_points(d) - 3))
        for _ in range(40):
            idx = rng.randrange(res.classes)
            mc, mt = res.class_mask(idx), res.witness_for_input(idx)
            assert oracle.scheme(d, canon, mc) == oracle.scheme(d, E, mt)


# ------------------------------------------------------------ regularity

def test_regularity_counts_table1():
    """Table 1 counts regular triangulations up to S3: all 18 orbits at
    d=3, 1278 of the 1279 flip-connected orbits at d=4.  The one non-regular
    orbit is fixed by the rotations of S3 (order 3) and has no certificate."""
    from paper_2604_09221_amd import regular as R

    _, orbs3 = orbit_table(3)
    assert all(R.is_regular(3, T) for _, T in orbs3.values())
    _, orbs4 = orbit_table(4)
    verdict = [(st, R.certificate(4, T)) for st, T in orbs4.values()]
    assert sum(w is not None for _, w in verdict) == 1278
    assert [st for st, w in verdict if w is None] == [3]


def test_regularity_certificates_are_exact():
    """Every certificate satisfies the local convexity inequalities in
    integers, and lifts (regular by construction) always get one."""
    from paper_2604_09221_amd import regular as R

    for d in (5, 7, 8, 12):
        for seed in range(3):
            E = I.lift_triangulation(d, seed, noise=1.0)
            w = R.certificate(d, E)
            assert w is not None and w.dtype == np.int64
            for a, b, c, e, al, be in R.edge_constraints(d, E):
                assert w[e] - (1 - al - be) * w[a] - al * w[b] - be * w[c] >= 1
    # the lower hull of the certificate's heights is T again (a different
    # derivation: the lifted triangles are faces of the lower hull, checked
    # with every lattice point strictly above each triangle's plane)
    d = 6
    E = I.lift_triangulation(d, 3, noise=1.0)
    w = R.certificate(d, E)
    pts = I.points(d)
    for t in K.triangles_of(d, [tuple(int(x) for x in e) for e in E]):
        (x0, y0), (x1, y1), (x2, y2) = t
        k0, k1, k2 = (pts.index(p) for p in t)
        det = (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0)
        for k, (x, y) in enumerate(pts):
            if k in (k0, k1, k2):
                continue
            # barycentric coordinates times det; plane value times det
            l1 = (x - x0) * (y2 - y0) - (y - y0) * (x2 - x0)
            l2 = (x1 - x0) * (y - y0) - (y1 - y0) * (x - x0)
            l0 = det - l1 - l2
            plane = l0 * w[k0] + l1 * w[k1] + l2 * w[k2]
            assert w[k] * det > plane if det > 0 else w[k] * det < plane
