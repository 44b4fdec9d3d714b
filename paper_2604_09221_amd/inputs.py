"""Seeded synthetic inputs: triangulations of d*Delta_2 and sign masks.

This module holds none of the scheme-extraction arithmetic.  It produces the
inputs that both the HIP path and the CPU oracle consume:

* ``standard_triangulation(d)`` -- the unimodular triangulation with edge
  directions (1,0), (0,1), (1,-1);
* ``lift_triangulation(d, seed, noise)`` -- the regular triangulation that is
  the lower hull of the lift h(i,j) = i^2 + i*j + j^2 + U[0, noise) (Sec. 2:
  regular = projection of the lower convex hull of a lift), computed with
  scipy and then verified with exact rational arithmetic;
* ``splitmix64(seed, n)`` -- the SplitMix64 generator (Steele, Lea, Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014), written from
  its published definition;
* ``random_masks(...)`` -- uniform sign masks (bit k = sigma(p_k), bit 0
  cleared so that sigma(0,0) = '+').

Lattice point order (a convention, not fixed by the paper):
k(i,j) = j(d+1) - j(j-1)/2 + i.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def n_points(d: int) -> int:
    return (d + 1) * (d + 2) // 2


def points(d: int):
    """Lattice points of d*Delta_2 in the project's bit order."""
    return [(i, j) for j in range(d + 1) for i in range(d + 1 - j)]


def standard_triangulation(d: int) -> np.ndarray:
    """Edge list (n_edges x 4: i0, j0, i1, j1) of the standard triangulation."""
    E = []
    for (i, j) in points(d):
        if i + 1 + j <= d:
            E.append((i, j, i + 1, j))
        if i + j + 1 <= d:
            E.append((i, j, i, j + 1))
        if i >= 1 and i - 1 + j + 1 <= d:
            E.append((i, j, i - 1, j + 1))
    return np.asarray(E, dtype=np.int32)


def lift_heights(d: int, seed: int, noise: float) -> np.ndarray:
    """h(i,j) = i^2 + i*j + j^2 + U[0, noise), one uniform draw per point in
    point order from numpy's default_rng(seed)."""
    u = np.random.default_rng(seed).random(n_points(d))
    P = points(d)
    return np.array([i * i + i * j + j * j for (i, j) in P], dtype=np.float64) + noise * u


def _above(a, b, c, p):
    """Exact sign of the orientation of lifted p against the plane of lifted
    a, b, c (positive = p above when (a,b,c) is counter-clockwise)."""
    (ax, ay, az), (bx, by, bz), (cx, cy, cz), (px, py, pz) = a, b, c, p
    m = [[bx - ax, by - ay, bz - az], [cx - ax, cy - ay, cz - az], [px - ax, py - ay, pz - az]]
    det = (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
           - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
           + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))
    return det


def lift_triangulation(d: int, seed: int, noise: float = 0.05) -> np.ndarray:
    """Regular triangulation of d*Delta_2 from the lower hull of the lift.

    Raises ValueError if the lower hull is not a unimodular triangulation or
    the lift is not generic (a point on a lower face's plane)."""
    from scipy.spatial import ConvexHull

    P = points(d)
    h = lift_heights(d, seed, noise)
    if d == 1:
        return np.asarray([(0, 0, 1, 0), (0, 0, 0, 1), (1, 0, 0, 1)], dtype=np.int32)
    X = np.array([(i, j, hz) for (i, j), hz in zip(P, h)], dtype=np.float64)
    hull = ConvexHull(X)
    tris = []
    for simplex, eq in zip(hull.simplices, hull.equations):
        if eq[2] < 0:  # outward normal points down: a lower face
            tris.append(tuple(int(s) for s in simplex))
    Q = [(Fraction(i), Fraction(j), Fraction(float(hz))) for (i, j), hz in zip(P, h)]
    edges = set()
    for (a, b, c) in tris:
        (ax, ay), (bx, by), (cx, cy) = P[a], P[b], P[c]
        det2 = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
        if abs(det2) != 1:
            raise ValueError(f"lower face {P[a]},{P[b]},{P[c]} is not unimodular (d={d}, seed={seed})")
        if det2 < 0:
            b, c = c, b
        # every other lifted point strictly above the face's plane: decided
        # in float64 where the margin is large, exactly otherwise
        u = X[b] - X[a]
        v = X[c] - X[a]
        w = X - X[a]
        det = (u[0] * (v[1] * w[:, 2] - v[2] * w[:, 1]) - u[1] * (v[0] * w[:, 2] - v[2] * w[:, 0])
               + u[2] * (v[0] * w[:, 1] - v[1] * w[:, 0]))
        for p in np.nonzero(det <= 1e-6)[0]:
            p = int(p)
            if p in (a, b, c):
                continue
            if _above(Q[a], Q[b], Q[c], Q[p]) <= 0:
                raise ValueError(f"lift not generic or hull wrong (d={d}, seed={seed})")
        for (u_, v_) in ((a, b), (b, c), (a, c)):
            edges.add((min(u_, v_), max(u_, v_)))
    if len(tris) != d * d:
        raise ValueError(f"{len(tris)} lower faces, expected {d * d}")
    E = sorted(edges)
    return np.asarray([(P[u][0], P[u][1], P[v][0], P[v][1]) for (u, v) in E], dtype=np.int32)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+n-1 of SplitMix64 started from state=seed."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def mask_words(d: int) -> int:
    """Words per mask: 1 x u32 (|A| <= 32), 1 x u64 (<= 64), 2 x u64."""
    n = n_points(d)
    return 1 if n <= 64 else 2


def random_masks(d: int, seed: int, n: int) -> np.ndarray:
    """n uniform masks (bit 0 cleared, bits >= |A| cleared) as an (n,2)
    uint64 array (lo, hi).  Masks of <= 64 bits use one output each, wider
    masks two consecutive outputs."""
    nA = n_points(d)
    out = np.zeros((n, 2), dtype=np.uint64)
    if nA <= 64:
        z = splitmix64(seed, n)
        keep = MASK64 if nA == 64 else np.uint64((1 << nA) - 1)
        out[:, 0] = z & keep
    else:
        z = splitmix64(seed, 2 * n).reshape(n, 2)
        out[:, 0] = z[:, 0]
        out[:, 1] = z[:, 1] & np.uint64((1 << (nA - 64)) - 1)
    out[:, 0] &= ~np.uint64(1)
    return out


def subsample_indices(seed: int, n: int, bits: int) -> np.ndarray:
    """n indices in [0, 2^bits) from SplitMix64 stream `seed`."""
    return splitmix64(seed, n) & np.uint64((1 << bits) - 1)


def pdep(value: int, select: int) -> int:
    """Deposit the low bits of `value` into the set bit positions of
    `select`, lowest first (the enumeration order of the masks)."""
    out, k = 0, 0
    pos = 0
    while select >> pos:
        if (select >> pos) & 1:
            if (value >> k) & 1:
                out |= 1 << pos
            k += 1
        pos += 1
    return out


def harnack_mask(d: int) -> int:
    """sigma(i,j) = '+' iff i and j are both even (the global flip of the
    classical Harnack distribution, so that sigma(0,0) = '+')."""
    m = 0
    for k, (i, j) in enumerate(points(d)):
        if not (i % 2 == 0 and j % 2 == 0):
            m |= 1 << k
    return m


def batched_degrees(n: int, seed: int = 0, lo: int = 4, hi: int = 12) -> np.ndarray:
    """Degree of slot t: lo + (SplitMix64(seed)_t mod (hi - lo + 1))."""
    return (lo + (splitmix64(seed, n) % np.uint64(hi - lo + 1))).astype(np.int64)


def masks128(masks2: np.ndarray) -> np.ndarray:
    """(n,2) uint64 masks -> flat int64 array, two words per mask (the
    layout of the multi-triangulation launch)."""
    return np.ascontiguousarray(masks2, dtype=np.uint64).reshape(-1).view(np.int64)
