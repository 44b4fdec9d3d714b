"""Independent checkers for the oracle (test code; shares nothing with
oracle/oracle.c or with the HIP path).

They rebuild the patchworked curve from (T, sigma) on their own and compute
quantities fixed by the mathematics rather than by Algorithm 1:

* ``betti``: Z/2 Betti numbers of the curve C as a 1-dimensional cell
  complex (0-cells = crossed edges of S, 1-cells = segments in the mixed
  triangles), by brute-force GF(2) elimination -- the homological route the
  paper contrasts with its algorithm (Sec. 1 footnote on polymake; Sec. 2,
  naive O(d^5) method);
* ``one_sided``: which curve components meet the line at infinity (the
  diamond boundary) an odd number of times;
* ``nesting_forest``: the oval nesting tree rebuilt oval by oval from
  two-sidedness and orientation parity, without the region adjacency graph;
* ``all_triangulations``: unimodular triangulations of d*Delta_2 by
  breadth-first search over flips (for small d).
"""
from __future__ import annotations

import itertools
from collections import deque


def points(d):
    return [(i, j) for j in range(d + 1) for i in range(d + 1 - j)]


def pidx(d, i, j):
    return j * (d + 1) - j * (j - 1) // 2 + i


def sigma_of(d, mask):
    return {(i, j): (mask >> pidx(d, i, j)) & 1 for (i, j) in points(d)}


def triangles_of(d, edges):
    """Unimodular 3-cliques of the edge graph (point tuples)."""
    E = set()
    for (a, b, c, e) in edges:
        E.add(((a, b), (c, e)))
        E.add(((c, e), (a, b)))
    nb = {}
    for (p, q) in E:
        nb.setdefault(p, set()).add(q)
    out = set()
    for (p, q) in E:
        for r in nb[p] & nb[q]:
            det = (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0])
            if abs(det) == 1:
                out.add(tuple(sorted((p, q, r))))
    return sorted(out)


QUAD = ((1, 1), (-1, 1), (1, -1), (-1, -1))


def diamond(d, edges):
    """Vertices, edges and triangles of T<> as coordinate tuples."""
    tris = set()
    for t in triangles_of(d, edges):
        for (ex, ey) in QUAD:
            tris.add(tuple(sorted((ex * p[0], ey * p[1]) for p in t)))
    E = set()
    for t in tris:
        for (p, q) in itertools.combinations(t, 2):
            E.add((min(p, q), max(p, q)))
    V = sorted({p for e in E for p in e})
    return V, sorted(E), sorted(tris)


def signs(d, mask, V):
    sg = sigma_of(d, mask)
    out = {}
    for (x, y) in V:
        s = sg[(abs(x), abs(y))]
        if x < 0:
            s += abs(x)
        if y < 0:
            s += abs(y)
        out[(x, y)] = s & 1
    return out


def on_boundary(d, p):
    return abs(p[0]) + abs(p[1]) == d


def neg(p):
    return (-p[0], -p[1])


def edge_class(d, e):
    """Representative of an edge of S: boundary edges are identified with
    their antipodal copies."""
    p, q = e
    if on_boundary(d, p) and on_boundary(d, q):
        f = (min(neg(p), neg(q)), max(neg(p), neg(q)))
        return min(e, f)
    return e


def vertex_class(d, p):
    if on_boundary(d, p):
        return min(p, neg(p))
    return p


def gf2_rank(rows):
    """Rank over GF(2) of rows given as Python-int bitsets."""
    basis = {}
    r = 0
    for v in rows:
        while v:
            h = v.bit_length() - 1
            if h in basis:
                v ^= basis[h]
            else:
                basis[h] = v
                r += 1
                break
    return r


def curve_cells(d, edges, mask):
    V, E, tris = diamond(d, edges)
    s = signs(d, mask, V)
    crossed = [e for e in E if s[e[0]] != s[e[1]]]
    cells0 = sorted({edge_class(d, e) for e in crossed})
    index0 = {c: k for k, c in enumerate(cells0)}
    segs = []
    for t in tris:
        ce = [edge_class(d, (min(p, q), max(p, q))) for (p, q) in itertools.combinations(t, 2)
              if s[p] != s[q]]
        assert len(ce) in (0, 2), "a triangle has 0 or 2 crossed edges"
        if ce:
            segs.append((index0[ce[0]], index0[ce[1]]))
    return V, E, tris, s, cells0, segs


def betti(d, edges, mask):
    """(b0(C), b1(C), b0(RP^2 minus C)) by GF(2) ranks."""
    V, E, tris, s, cells0, segs = curve_cells(d, edges, mask)
    rank = gf2_rank([(1 << a) ^ (1 << b) for (a, b) in segs])
    b0 = len(cells0) - rank
    b1 = len(segs) - rank
    # complement: vertices of S, non-crossed edges of S
    vcls = sorted({vertex_class(d, p) for p in V})
    vi = {c: k for k, c in enumerate(vcls)}
    ecls = sorted({edge_class(d, e) for e in E if s[e[0]] == s[e[1]]})
    rows = []
    for (p, q) in ecls:
        a, b = vi[vertex_class(d, p)], vi[vertex_class(d, q)]
        if a != b:
            rows.append((1 << a) ^ (1 << b))
    regions = len(vcls) - gf2_rank(rows)
    return b0, b1, regions


def _components(n, pairs):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for (a, b) in pairs:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    return [find(x) for x in range(n)]


def curve_components(d, edges, mask):
    """Curve components as lists of crossed-edge classes (0-cells)."""
    V, E, tris, s, cells0, segs = curve_cells(d, edges, mask)
    lab = _components(len(cells0), segs)
    comps = {}
    for k, r in enumerate(lab):
        comps.setdefault(r, []).append(cells0[k])
    return list(comps.values()), V, E, s


def one_sided(d, edges, mask):
    """Per curve component: True iff it meets the diamond boundary (the line
    at infinity) in an odd number of points."""
    comps, V, E, s = curve_components(d, edges, mask)
    out = []
    for c in comps:
        nb = sum(1 for (p, q) in c if on_boundary(d, p) and on_boundary(d, q))
        out.append(nb % 2 == 1)
    return out


def nesting_forest(d, edges, mask):
    """Nesting forest of the ovals, rebuilt per oval.

    For an oval O, the T<> edges not crossed by O (label 0) and the
    antipodal pairs (label 1) connect the vertices of A<> into exactly two
    classes: the disk inside O and the Moebius band outside it.  The outside
    class is the one carrying a cycle with an odd number of antipodal jumps.
    O' lies inside O iff the endpoints of O''s crossed edges lie in O's
    inside class.  The parent of O' is its innermost enclosing oval."""
    comps, V, E, s = curve_components(d, edges, mask)
    ovals = []
    for c in comps:
        nb = sum(1 for (p, q) in c if on_boundary(d, p) and on_boundary(d, q))
        if nb % 2 == 0:
            ovals.append(c)
    vi = {p: k for k, p in enumerate(V)}
    anti = [(vi[p], vi[neg(p)]) for p in V if on_boundary(d, p) and p < neg(p)]
    inside = []
    for O in ovals:
        cut = set()
        for e in O:
            cut.add(e)
            p, q = e
            if on_boundary(d, p) and on_boundary(d, q):
                cut.add((min(neg(p), neg(q)), max(neg(p), neg(q))))
        adj = [[] for _ in V]
        for (p, q) in E:
            if (p, q) in cut:
                continue
            adj[vi[p]].append((vi[q], 0))
            adj[vi[q]].append((vi[p], 0))
        for (a, b) in anti:
            adj[a].append((b, 1))
            adj[b].append((a, 1))
        col = [-1] * len(V)
        cls = [-1] * len(V)
        ncls = 0
        odd = []
        for s0 in range(len(V)):
            if col[s0] >= 0:
                continue
            col[s0] = 0
            cls[s0] = ncls
            dq = deque([s0])
            bad = False
            while dq:
                v = dq.popleft()
                for (u, w) in adj[v]:
                    if col[u] < 0:
                        col[u] = col[v] ^ w
                        cls[u] = ncls
                        dq.append(u)
                    elif col[u] != col[v] ^ w:
                        bad = True
            odd.append(bad)
            ncls += 1
        assert ncls == 2, f"an oval should cut RP^2 in two, got {ncls}"
        assert sorted(odd) == [False, True], "exactly one side is non-orientable"
        inside.append((cls, odd.index(False)))
    n = len(ovals)
    contains = [[False] * n for _ in range(n)]
    for a in range(n):
        cls, ins = inside[a]
        for b in range(n):
            if a == b:
                continue
            p, q = ovals[b][0]
            assert cls[vi[p]] == cls[vi[q]]
            contains[a][b] = cls[vi[p]] == ins
    depth = [sum(contains[a][b] for a in range(n)) for b in range(n)]
    children = [[] for _ in range(n)]
    roots = []
    for b in range(n):
        enc = [a for a in range(n) if contains[a][b]]
        if not enc:
            roots.append(b)
        else:
            par = max(enc, key=lambda a: depth[a])
            children[par].append(b)

    def build(v):
        return [build(c) for c in children[v]]

    return [build(r) for r in roots]


# ---- triangulations by flips ----

def _tri_set(d, edges):
    return frozenset((min((a, b), (c, e)), max((a, b), (c, e))) for (a, b, c, e) in edges)


def _to_edges(es):
    return [(p[0], p[1], q[0], q[1]) for (p, q) in sorted(es)]


def flips(d, es):
    """All triangulations one flip away: an interior edge whose two
    triangles form a parallelogram is replaced by the other diagonal."""
    tris = triangles_of(d, _to_edges(es))
    by_edge = {}
    for t in tris:
        for (p, q) in itertools.combinations(t, 2):
            by_edge.setdefault((p, q), []).append(t)
    out = []
    for e, ts in by_edge.items():
        if len(ts) != 2:
            continue
        p, q = e
        r1 = [x for x in ts[0] if x not in e][0]
        r2 = [x for x in ts[1] if x not in e][0]
        if (p[0] + q[0] == r1[0] + r2[0]) and (p[1] + q[1] == r1[1] + r2[1]):
            ne = (min(r1, r2), max(r1, r2))
            out.append(frozenset((es - {e}) | {ne}))
    return out


def all_triangulations(d, start_edges):
    """Every unimodular triangulation of d*Delta_2 reachable by flips."""
    s0 = _tri_set(d, start_edges)
    seen = {s0}
    dq = deque([s0])
    while dq:
        t = dq.popleft()
        for u in flips(d, t):
            if u not in seen:
                seen.add(u)
                dq.append(u)
    return [_to_edges(t) for t in seen]


# ---- the S3 action on barycentric coordinates (i, j, d-i-j) ----

def s3_maps(d):
    out = []
    for perm in itertools.permutations(range(3)):
        def f(p, perm=perm):
            b = (p[0], p[1], d - p[0] - p[1])
            c = tuple(b[perm[k]] for k in range(3))
            return (c[0], c[1])
        out.append(f)
    return out


def act_s3(d, edges, mask, f):
    E2 = [(*f((a, b)), *f((c, e))) for (a, b, c, e) in edges]
    sg = sigma_of(d, mask)
    m2 = 0
    for p, v in sg.items():
        if v:
            q = f(p)
            m2 |= 1 << pidx(d, q[0], q[1])
    return E2, m2


def affine_flip(d, mask, a, b, c):
    """sigma -> sigma + a + b*i + c*j (mod 2)."""
    m2 = 0
    for (i, j), v in sigma_of(d, mask).items():
        if (v + a + b * i + c * j) & 1:
            m2 |= 1 << pidx(d, i, j)
    return m2
