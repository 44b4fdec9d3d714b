"""Oracle of the triangulation search steps (Sec. 3: random flips of
unimodular triangulations, symmetric triangulations, the per-triangulation
objectives of simulated annealing and its accept rule).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the device calls; the
product never imports it.  Plain Python on edge sets, one triangulation and
one move at a time, written from the definitions:

* a flip replaces an interior edge ab, whose two triangles abc and abe form
  a parallelogram (c + e = a + b), by the other diagonal ce;
* a move draws r1, r2 from the SplitMix64 finaliser F (Steele, Lea, Flood
  2014) as r_k = F(seed ^ F(w * 0x100000001B3 + 2 step + k)); a = r1 mod |A|,
  b = the (r2 mod deg a)-th neighbour of a by point index, and ab is flipped
  if possible; in symmetric mode (mirror s(i, j) = (j, i)) an edge fixed by
  s is flipped alone, otherwise ab and s(ab) are flipped together when both
  are flippable and no triangle contains both;
* objectives: the number of distinct codes; the number of codes whose
  scheme has p ovals at odd depth and n at even depth;
* accept: the proposal replaces the current state if its score is not lower,
  else if the 24-bit draw u = F(seed ^ F(chain * 0x100000001B3 + step)) >> 40
  is below accept[k - 1], k the score drop.
"""
from __future__ import annotations

M64 = (1 << 64) - 1


def mix(z: int) -> int:
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def draw(seed: int, w: int, c: int) -> int:
    return mix(seed ^ mix((w * 0x100000001B3 + c) & M64))


def points(d):
    return [(i, j) for j in range(d + 1) for i in range(d + 1 - j)]


class Tri:
    """A triangulation as a set of edges between lattice points."""

    def __init__(self, d, edges):
        self.d = d
        self.pts = points(d)
        self.idx = {p: k for k, p in enumerate(self.pts)}
        self.E = set()
        for a, b, c, e in edges:
            p, q = self.idx[(int(a), int(b))], self.idx[(int(c), int(e))]
            self.E.add((min(p, q), max(p, q)))

    def nbrs(self, p):
        return sorted([q for (x, q) in self.E if x == p] + [x for (x, q) in self.E if q == p])

    def has(self, p, q):
        return (min(p, q), max(p, q)) in self.E

    def apexes(self, a, b):
        """(left, right) apex of edge ab: common neighbours c with
        det(b - a, c - a) = +1 / -1 (None where missing)."""
        (ia, ja), (ib, jb) = self.pts[a], self.pts[b]
        left = right = None
        for c in set(self.nbrs(a)) & set(self.nbrs(b)):
            ic, jc = self.pts[c]
            det = (ib - ia) * (jc - ja) - (jb - ja) * (ic - ia)
            if det == 1:
                left = c
            elif det == -1:
                right = c
        return left, right

    def flippable(self, a, b):
        if not self.has(a, b):
            return None
        c, e = self.apexes(a, b)
        if c is None or e is None:
            return None
        pa, pb, pc, pe = (self.pts[x] for x in (a, b, c, e))
        if pc[0] + pe[0] == pa[0] + pb[0] and pc[1] + pe[1] == pa[1] + pb[1]:
            return c, e
        return None

    def flip(self, a, b, c, e):
        self.E.remove((min(a, b), max(a, b)))
        self.E.add((min(c, e), max(c, e)))

    def mirror(self, p):
        i, j = self.pts[p]
        return self.idx[(j, i)]

    def edges(self):
        return sorted((*self.pts[p], *self.pts[q]) for p, q in self.E)


def flip_walk(d, edges, steps, symmetric, seed, w, step0=0):
    """The walk of triangulation number w: returns (edges, moves made)."""
    T = Tri(d, edges)
    nA = len(T.pts)
    moves = 0
    for s in range(steps):
        c0 = 2 * (step0 + s)
        r1, r2 = draw(seed, w, c0), draw(seed, w, c0 + 1)
        a = r1 % nA
        nb = T.nbrs(a)
        if not nb:
            continue
        b = nb[r2 % len(nb)]
        f = T.flippable(a, b)
        if f is None:
            continue
        if not symmetric:
            T.flip(a, b, *f)
            moves += 1
            continue
        sa, sb = T.mirror(a), T.mirror(b)
        if {sa, sb} == {a, b}:
            T.flip(a, b, *f)
            moves += 1
            continue
        g = T.flippable(sa, sb)
        if g is None:
            continue
        # no triangle holds both edges: s(ab) is not a side of ab's quadrilateral
        if {sa, sb} in ({a, f[0]}, {b, f[0]}, {a, f[1]}, {b, f[1]}):
            continue
        T.flip(a, b, *f)
        T.flip(sa, sb, *g)
        moves += 1
    return T.edges(), moves


def is_symmetric(d, edges):
    E = {tuple(e) for e in map(tuple, edges)}
    norm = {tuple(sorted([(a, b), (c, e)])) for a, b, c, e in E}
    return {tuple(sorted([(b, a), (e, c)])) for (a, b), (c, e) in norm} == norm


def code_pn(code: int):
    """(p, n): ovals at odd depth (outermost = 1) and at even depth, read
    from the code's bit string (a '1' opens a node, a '0' closes it)."""
    lo = code & ((1 << 127) - 1)
    bits = bin(lo)[3:]
    depth = p = n = 0
    for ch in bits:
        if ch == "1":
            depth += 1
            if depth % 2:
                p += 1
            else:
                n += 1
        else:
            depth -= 1
    return p, n


def objective(codes, mode, target=(0, 0)):
    """Score of one triangulation's list of codes (ints; 0 = failed)."""
    good = [c for c in codes if c != 0]
    if mode == 0:
        return len(set(good))
    return sum(1 for c in good if code_pn(c) == tuple(target))


def accept(score_cur, score_prop, table, seed, chain, step):
    if score_prop >= score_cur:
        return True
    k = int(score_cur - score_prop)
    u = draw(seed, chain, step) >> 40
    return 1 <= k <= len(table) and u < table[k - 1]
