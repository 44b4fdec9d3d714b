"""Orbit-reduced exhaustive sweeps (Sec. 3, Table 1).

Two symmetries leave the real scheme unchanged:
* (Z/2)^3 on sign distributions, sigma -> sigma + a + b i + c j (mod 2): it
  acts freely, so sweeping one representative per class (sigma fixed to '+'
  at three points of distinct parity classes, ``pw_class_fixed_bits``)
  covers every distribution, each class standing for 8;
* S3 on triangulations, permuting the barycentric coordinates (i, j,
  d-i-j) of both T and sigma: one member of each orbit of triangulations
  stands for the 6 (3 for those fixed by a transposition, 1 for the fully
  symmetric) whose sweeps realise the same schemes.

``orbit_sweep`` canonicalises T (``pw_tri_canonical``), sweeps the (Z/2)^3
classes of the canonical member on the GPU (``enumerate_range``) and
returns the class histogram with the multiplicities that turn it into the
histogram of every (T', sigma) pair of the orbit.  This module only
arranges the calls; the canonical form, the class representatives and the
sweep are the library's.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import inputs as I
from . import patchwork as pw


@dataclass
class OrbitSweep:
    d: int
    canonical_edges: np.ndarray     # (n, 4) int16, the swept member of the orbit
    perm_index: int                 # S3 permutation taking the input T to it
    stabilizer: int                 # permutations fixing T: 1, 2, 3 or 6
    fixed_zero_bits: int            # the three class-representative points
    classes: int                    # class representatives swept
    hist: dict = field(default_factory=dict)   # code -> (count of classes, smallest class index)

    @property
    def orbit_size(self) -> int:
        return 6 // self.stabilizer

    @property
    def pairs_covered(self) -> int:
        """(T', sigma) pairs of the whole orbit the sweep classifies: every
        class stands for 8 sign distributions, for each of the orbit's
        triangulations."""
        return 8 * self.orbit_size * self.classes

    def class_mask(self, index: int) -> int:
        """The sign mask (of the canonical member) of class `index`."""
        free = ((1 << I.n_points(self.d)) - 1) & ~self.fixed_zero_bits
        return I.pdep(int(index), free)

    def witness_for_input(self, index: int) -> int:
        """A mask of the INPUT triangulation with the same scheme as class
        `index` of the canonical member (sigma_T = sigma_C o pi)."""
        m = self.class_mask(index)
        pm = pw.point_map(self.d, self.perm_index)
        out = 0
        for p in range(I.n_points(self.d)):
            if (m >> int(pm[p])) & 1:
                out |= 1 << p
        return out

    def full_counts(self) -> dict:
        """code -> number of sign distributions of any one triangulation of
        the orbit with that scheme (8 per class)."""
        return {c: 8 * n for c, (n, _) in self.hist.items()}


def orbit_sweep(d: int, edges, capacity: int = 4096, specialize: bool = True, first: int = 0, count=None,
                stream=None) -> OrbitSweep:
    """Sweep every (Z/2)^3 class of the canonical member of T's S3 orbit
    (or the class range [first, first + count))."""
    canon, k, stab = pw.canonical(d, edges)
    fixed = pw.class_fixed_bits(d)
    n_classes = 1 << (I.n_points(d) - 3)
    if count is None:
        count = n_classes - first
    tri = pw.Triangulation(d, canon)
    if specialize and d <= 9:
        tri.specialize()
    h = pw.Histogram(capacity)
    tri.enumerate_range(first, count, h, fixed_zero_bits=fixed, stream=stream)
    res = OrbitSweep(d, canon, k, stab, fixed, count, h.read())
    if tri.errors() != 0:
        raise pw.PatchworkError(pw.PW_ERR_INTERNAL, "device consistency check failed in the orbit sweep")
    return res
