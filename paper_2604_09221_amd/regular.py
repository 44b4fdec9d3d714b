"""Regularity of a unimodular triangulation (Sec. 2: Viro's patchworking
starts from a convex, i.e. regular, triangulation; Table 1 counts regular
triangulations).

T is regular iff some heights w : A -> R make the piecewise-linear function
that interpolates w on the triangles of T strictly convex: across every
interior edge ab with apexes c and e, the lifted e lies strictly above the
plane through the lifted a, b, c.  Writing e - a = alpha (b - a) + beta (c - a)
(alpha, beta integers, since abc is unimodular), the condition is

    w(e) - w(a) - alpha (w(b) - w(a)) - beta (w(c) - w(a)) >= 1

after scaling.  A piecewise-linear function on a convex domain that is
locally convex across every interior edge is convex, so these constraints
are exactly regularity.  The linear program is solved in floating point
(HiGHS); a feasible answer is turned into integer heights and every
constraint is re-checked in exact integer arithmetic, so a "regular"
verdict always comes with a verified certificate.  Host-side; not a step of
Alg. 1.
"""
from __future__ import annotations

import numpy as np

from . import inputs as I


def edge_constraints(d: int, edges):
    """Rows (a, b, c, e, alpha, beta) for every interior edge ab with
    apexes c (left) and e (right), point indices into A."""
    pts = I.points(d)
    index = {p: k for k, p in enumerate(pts)}
    nbr = {p: set() for p in pts}
    E = [((int(a), int(b)), (int(c), int(e))) for a, b, c, e in np.asarray(edges).reshape(-1, 4)]
    for p, q in E:
        nbr[p].add(q)
        nbr[q].add(p)
    rows = []
    for p, q in E:
        vx, vy = q[0] - p[0], q[1] - p[1]
        left = right = None
        for c in nbr[p] & nbr[q]:
            det = vx * (c[1] - p[1]) - vy * (c[0] - p[0])
            if det == 1:
                left = c
            elif det == -1:
                right = c
        if left is None or right is None:
            continue  # boundary edge
        # e - a = alpha (b - a) + beta (c - a), with det(b - a, c - a) = 1
        ex, ey = right[0] - p[0], right[1] - p[1]
        cx, cy = left[0] - p[0], left[1] - p[1]
        alpha = ex * cy - ey * cx
        beta = vx * ey - vy * ex
        rows.append((index[p], index[q], index[left], index[right], alpha, beta))
    return rows


def _matrix(n, rows):
    A = np.zeros((len(rows), n), dtype=np.int64)
    for r, (a, b, c, e, al, be) in enumerate(rows):
        A[r, e] += 1
        A[r, a] -= 1 - al - be
        A[r, b] -= al
        A[r, c] -= be
    return A


def certificate(d: int, edges):
    """Integer heights (numpy int64, one per lattice point) certifying that
    T is regular, or None if T is not regular."""
    from scipy.optimize import linprog

    rows = edge_constraints(d, edges)
    n = I.n_points(d)
    A = _matrix(n, rows)
    if len(rows) == 0:
        return np.zeros(n, dtype=np.int64)
    # A w >= 1  <=>  -A w <= -1; w(0,0) pinned to 0 (heights are defined up
    # to adding an affine function)
    bounds = [(0, 0)] + [(None, None)] * (n - 1)
    res = linprog(np.zeros(n), A_ub=-A.astype(float), b_ub=-np.ones(len(rows)), bounds=bounds, method="highs")
    if res.status == 2:
        return None
    if res.status != 0:
        raise RuntimeError(f"regularity LP failed: {res.message}")
    w = np.asarray(res.x, dtype=float)
    # scale so that rounding each height moves every constraint by less than
    # half its margin, then check exactly
    s = float(np.abs(A).sum(axis=1).max())
    for scale in (2 * s, 8 * s, 64 * s):
        wi = np.rint(w * scale).astype(np.int64)
        if (A @ wi >= 1).all():
            return wi
    raise RuntimeError("regularity LP solution could not be certified in integers")


def is_regular(d: int, edges) -> bool:
    return certificate(d, edges) is not None
