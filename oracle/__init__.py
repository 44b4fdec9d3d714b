"""CPU oracle for real-scheme extraction -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference for Algorithm 1 of "Fast Isotopy
Computation for T-Curves" (Sec. 2).  The arithmetic lives in ``oracle.c``
(plain C, breadth-first search, string codes); this module only builds and
loads it and decodes its scheme codes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never imports it and shares no code with it.

Scheme code (the paper fixes no encoding for "canonical form", Alg. 1 last
step; this is the project's choice): for a node v of the rooted region tree,
``c(v) = '1' + concat(sorted(c(children), descending)) + '0'``; ``W`` is the
concatenation of the sorted codes of the root's children; the code is the
128-bit integer ``2**len(W) + int(W, 2)``, with bit 127 set iff d is odd (the
pseudo-line J, Sec. 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

J_BIT = 1 << 127


def build(force: bool = False) -> str:
    """Compile oracle.c with plain gcc -O2 (no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_last_error.restype = ctypes.c_char_p
        L.oracle_validate.argtypes = [ctypes.c_int, i32p, ctypes.c_int]
        L.oracle_triangles.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p]
        L.oracle_diamond_sizes.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p]
        L.oracle_scheme.argtypes = [ctypes.c_int, i32p, ctypes.c_int, u64p, u64p, i32p]
        L.oracle_scheme_many.argtypes = [ctypes.c_int, i32p, ctypes.c_int, u64p, ctypes.c_int64, u64p,
                                         ctypes.c_int]
        L.oracle_point_index.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_diamond_signs.argtypes = [ctypes.c_int, i32p, ctypes.c_int, u64p, i32p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _edges_arr(edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 4))
    return e


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _check(rc):
    if rc != 0:
        raise OracleError(f"oracle error {rc}: {lib().oracle_last_error().decode()}")


def validate(d: int, edges) -> None:
    e = _edges_arr(edges)
    _check(lib().oracle_validate(d, _p(e, ctypes.c_int32), len(e)))


def triangles(d: int, edges) -> np.ndarray:
    """The d*d triangles of T as point-index triples."""
    e = _edges_arr(edges)
    out = np.zeros((d * d, 3), dtype=np.int32)
    _check(lib().oracle_triangles(d, _p(e, ctypes.c_int32), len(e), _p(out, ctypes.c_int32)))
    return out


def diamond_sizes(d: int, edges):
    e = _edges_arr(edges)
    out = np.zeros(3, dtype=np.int32)
    _check(lib().oracle_diamond_sizes(d, _p(e, ctypes.c_int32), len(e), _p(out, ctypes.c_int32)))
    return tuple(int(x) for x in out)


def _masks2(masks) -> np.ndarray:
    """Any of: python ints, uint32/uint64 array (one word per mask), or an
    (n,2) uint64 array -> contiguous (n,2) uint64."""
    if isinstance(masks, np.ndarray) and masks.ndim == 2:
        return np.ascontiguousarray(masks.astype(np.uint64))
    if isinstance(masks, np.ndarray):
        out = np.zeros((masks.shape[0], 2), dtype=np.uint64)
        out[:, 0] = masks.astype(np.uint64)
        return out
    ms = list(masks)
    out = np.zeros((len(ms), 2), dtype=np.uint64)
    for k, m in enumerate(ms):
        m = int(m)
        out[k, 0] = m & 0xFFFFFFFFFFFFFFFF
        out[k, 1] = (m >> 64) & 0xFFFFFFFFFFFFFFFF
    return out


def scheme(d: int, edges, mask: int, with_info: bool = False):
    """Code of one pair (T, sigma) as a Python int (and the counts
    components, regions, ovals, root region, max depth)."""
    e = _edges_arr(edges)
    m = _masks2([mask])
    code = np.zeros(2, dtype=np.uint64)
    info = np.zeros(5, dtype=np.int32)
    _check(lib().oracle_scheme(d, _p(e, ctypes.c_int32), len(e), _p(m, ctypes.c_uint64),
                               _p(code, ctypes.c_uint64), _p(info, ctypes.c_int32)))
    c = int(code[0]) | (int(code[1]) << 64)
    if with_info:
        return c, dict(zip(("components", "regions", "ovals", "root", "max_depth"), (int(x) for x in info)))
    return c


def scheme_many(d: int, edges, masks, threads: int = 1) -> np.ndarray:
    """Codes of many masks for one triangulation, as an (n,2) uint64 array
    (lo, hi words)."""
    e = _edges_arr(edges)
    m = _masks2(masks)
    codes = np.zeros_like(m)
    _check(lib().oracle_scheme_many(d, _p(e, ctypes.c_int32), len(e), _p(m, ctypes.c_uint64), len(m),
                                    _p(codes, ctypes.c_uint64), int(threads)))
    return codes


def diamond_signs(d: int, edges, mask: int) -> dict:
    """{(x, y): sign} on A<> as the oracle extends sigma (eq. (signs))."""
    e = _edges_arr(edges)
    m = _masks2([mask])
    nV = 2 * d * d + 2 * d + 1
    out = np.zeros((nV, 3), dtype=np.int32)
    _check(lib().oracle_diamond_signs(d, _p(e, ctypes.c_int32), len(e), _p(m, ctypes.c_uint64),
                                      _p(out, ctypes.c_int32)))
    return {(int(x), int(y)): int(s) for (x, y, s) in out}


def point_index(d: int, i: int, j: int) -> int:
    return int(lib().oracle_point_index(d, i, j))


# ---- decoding of scheme codes (display and features) ----

def code_int(lo, hi) -> int:
    return int(lo) | (int(hi) << 64)


def has_J(code: int) -> bool:
    return bool(code & J_BIT)


def word(code: int) -> str:
    """The scheme word W of a code (bit string, most significant first)."""
    c = code & (J_BIT - 1)
    if c <= 0:
        raise ValueError("not a scheme code")
    return bin(c)[3:]


def n_ovals(code: int) -> int:
    return len(word(code)) // 2


def parse_tree(w: str):
    """The Dyck word W as a forest: list of children lists (recursive)."""
    stack = [[]]
    for ch in w:
        if ch == "1":
            node = []
            stack[-1].append(node)
            stack.append(node)
        else:
            stack.pop()
    assert len(stack) == 1
    return stack[0]


def oval_depths(code: int):
    """Depth of each oval (outermost = 1), in word order."""
    out, bal = [], 0
    for ch in word(code):
        if ch == "1":
            bal += 1
            out.append(bal)
        else:
            bal -= 1
    return out


def rohlin_viro(code: int) -> str:
    """Display form, e.g. '<J + 1<2> + 5>' ('+' stands for the disjoint
    union).  k identical empty ovals are written as the integer k."""

    def fmt(forest):
        parts = []
        leaves = sum(1 for t in forest if not t)
        groups = {}
        order = []
        for t in forest:
            if t:
                key = fmt(t)
                if key not in groups:
                    groups[key] = 0
                    order.append(key)
                groups[key] += 1
        for key in order:
            k = groups[key]
            parts.append((f"{k}" if k > 1 else "1") + f"<{key}>")
        if leaves:
            parts.append(str(leaves))
        return " + ".join(parts) if parts else "0"

    body = fmt(parse_tree(word(code)))
    if has_J(code):
        body = "J" if body == "0" else "J + " + body
    return f"<{body}>"


def code_from_forest(forest, odd: bool) -> int:
    """Encode a forest (children lists) with the canonical rule above."""

    def c(node):
        return "1" + "".join(sorted((c(ch) for ch in node), reverse=True)) + "0"

    w = "".join(sorted((c(t) for t in forest), reverse=True))
    v = int("1" + w, 2)
    return v | (J_BIT if odd else 0)
