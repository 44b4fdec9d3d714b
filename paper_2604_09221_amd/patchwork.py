"""Python binding of libpatchwork.so (ctypes; argument marshalling only).

Every computation runs in the library's HIP kernels.  PyTorch provides the
device buffers and the current stream; this module only passes pointers and
sizes through the C-ABI declared in ``include/patchwork.h``.  There is no
fallback: if the library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpatchwork.so")

PW_OK = 0
PW_ERR_ARG = -1
PW_ERR_TRI = -2
PW_ERR_HIP = -3
PW_ERR_RANGE = -4
PW_ERR_HIST_FULL = -5
PW_ERR_INTERNAL = -6

J_BIT = 1 << 127

_lib = None


class MultiConfig(ctypes.Structure):
    """Launch shape of patchwork_scheme_batch_multi (pw_multi_config)."""
    _fields_ = [("chunk", ctypes.c_int32), ("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lane_groups", ctypes.c_uint32)]


def lane_groups_code(groups: dict) -> int:
    """pw_multi_config.lane_groups from {degree: lanes per mask (1, 2 or 4)}."""
    code = 0
    for d, g in groups.items():
        code |= {1: 0, 2: 1, 4: 2}[int(g)] << (2 * int(d))
    return code


def lane_groups_of(code: int) -> dict:
    """{degree: lanes per mask} for the degrees with more than one lane."""
    return {d: {1: 2, 2: 4}[(code >> (2 * d)) & 3] for d in range(16) if (code >> (2 * d)) & 3}


# the library's lane groups when no configuration is passed
# (PW_MULTI_DEFAULT_LANE_GROUPS: four lanes per mask for degrees 11 and 12)
DEFAULT_LANE_GROUPS = lane_groups_code({11: 4, 12: 4})


class PatchworkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"patchwork error {status}: {msg}")
        self.status = status


def lib():
    """Load libpatchwork.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    i32p = ctypes.POINTER(ctypes.c_int32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.pw_last_error.restype = ctypes.c_char_p
    L.pw_version.restype = i32
    L.pw_mask_bytes.argtypes = [i32]
    L.pw_mask_bytes.restype = i32
    L.pw_tri_create.argtypes = [i32, ctypes.POINTER(ctypes.c_int16), i32, ctypes.POINTER(vp)]
    L.pw_tri_destroy.argtypes = [vp]
    L.pw_tri_info.argtypes = [vp, i32p, i32p, i32p, i32p, i32p]
    L.pw_tri_errors.argtypes = [vp, u32p]
    L.patchwork_scheme_batch.argtypes = [vp, vp, i64, vp, vp]
    L.pw_hist_create.argtypes = [i32, ctypes.POINTER(vp)]
    L.pw_hist_reset.argtypes = [vp, vp]
    L.pw_hist_read.argtypes = [vp, u64p, u64p, u64p, i32, i32p]
    L.pw_hist_destroy.argtypes = [vp]
    L.patchwork_scheme_histogram.argtypes = [vp, vp, i64, u64, vp, vp]
    L.patchwork_scheme_codes_histogram.argtypes = [vp, vp, i64, u64, vp, vp, vp]
    L.patchwork_scheme_enumerate_range.argtypes = [vp, u64, u64, u64p, vp, vp]
    L.patchwork_scheme_sweep_graph.argtypes = [vp, u64, u64, u64, u64p, vp, vp]
    L.pw_tri_specialize.argtypes = [vp]
    i16p = ctypes.POINTER(ctypes.c_int16)
    L.pw_jit_source.argtypes = [i32, i16p, i32, ctypes.c_char_p, i64, ctypes.POINTER(ctypes.c_int64)]
    L.pw_jit_compile.argtypes = [i32, i16p, i32, ctypes.POINTER(ctypes.c_int64)]
    L.patchwork_scheme_batch_multi.argtypes = [ctypes.POINTER(vp), i32, vp, ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(vp), vp, ctypes.POINTER(MultiConfig), vp]
    L.patchwork_scheme_batch_multi_noalloc.argtypes = L.patchwork_scheme_batch_multi.argtypes
    L.pw_tri_program.argtypes = [vp, u32p, i32, i32p]
    L.pw_tri_group_program.argtypes = [vp, i32, u32p, i32, i32p]
    L.pw_tri_canonical.argtypes = [i32, i16p, i32, i16p, i32p, i32p]
    L.pw_point_map.argtypes = [i32, i32, i32p]
    L.pw_class_fixed_bits.argtypes = [i32, u64p]
    L.pw_program_words.argtypes = [i32]
    L.pw_adjacency_from_edges.argtypes = [i32, i16p, i32, u64p]
    L.pw_edges_from_adjacency.argtypes = [i32, u64p, i16p, i32, i32p]
    L.pw_flip_walk.argtypes = [i32, vp, i64, i32, i32, u64, u64, vp, vp]
    L.pw_build_programs.argtypes = [i32, vp, i64, vp, vp, vp]
    L.patchwork_scheme_programs.argtypes = [i32, vp, i64, vp, i64, vp, vp, vp, vp]
    L.pw_tri_objective.argtypes = [i32, vp, i64, i32, i32, i32, i32, vp, i32, vp, vp]
    L.pw_anneal_accept.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, i32, u64, u64, vp, vp]
    for name in ("pw_tri_program", "pw_tri_group_program", "pw_tri_canonical", "pw_point_map", "pw_class_fixed_bits", "pw_program_words",
                 "pw_adjacency_from_edges", "pw_edges_from_adjacency", "pw_flip_walk", "pw_build_programs",
                 "patchwork_scheme_programs", "pw_tri_objective", "pw_anneal_accept"):
        getattr(L, name).restype = i32
    for name in ("pw_tri_create", "pw_tri_destroy", "pw_tri_info", "pw_tri_errors", "patchwork_scheme_batch",
                 "pw_hist_create", "pw_hist_reset", "pw_hist_read", "pw_hist_destroy",
                 "patchwork_scheme_histogram", "patchwork_scheme_codes_histogram", "patchwork_scheme_enumerate_range", "patchwork_scheme_sweep_graph",
                 "patchwork_scheme_batch_multi", "patchwork_scheme_batch_multi_noalloc",
                 "pw_tri_specialize", "pw_jit_source", "pw_jit_compile"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def check(status):
    if status != PW_OK:
        raise PatchworkError(status, lib().pw_last_error().decode())


def mask_bytes(d: int) -> int:
    n = lib().pw_mask_bytes(d)
    if n < 0:
        raise PatchworkError(n, "degree out of range")
    return n


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def mask_tensor(masks2: np.ndarray, d: int, device="cuda"):
    """Host (n,2) uint64 masks -> a device tensor in the library's mask
    layout for degree d (int32 / int64 / int64 pairs)."""
    import torch

    nb = mask_bytes(d)
    m = np.ascontiguousarray(masks2, dtype=np.uint64).reshape(-1, 2)
    if nb == 4:
        host = m[:, 0].astype(np.uint32).view(np.int32)
    elif nb == 8:
        host = m[:, 0].view(np.int64)
    else:
        host = m.view(np.int64).reshape(-1)
    return torch.from_numpy(np.ascontiguousarray(host)).to(device)


def codes_to_ints(codes) -> list:
    """(n,2) int64 tensor/array of (lo, hi) words -> Python ints."""
    a = codes.cpu().numpy() if hasattr(codes, "cpu") else np.asarray(codes)
    a = a.view(np.uint64).reshape(-1, 2)
    return [int(lo) | (int(hi) << 64) for lo, hi in a]


class Triangulation:
    """A validated triangulation handle (pw_tri_create)."""

    def __init__(self, d: int, edges):
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int16).reshape(-1, 4))
        h = ctypes.c_void_p()
        check(lib().pw_tri_create(int(d), e.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)), len(e),
                                  ctypes.byref(h)))
        self.handle = h
        self.d = int(d)

    def close(self):
        if self.handle:
            lib().pw_tri_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        v = [ctypes.c_int32() for _ in range(5)]
        check(lib().pw_tri_info(self.handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(("d", "n_points", "n_vertices", "n_diamond_edges", "n_antipodal_pairs"),
                        (x.value for x in v)))

    def specialize(self):
        """Build and load kernels specialised to this triangulation."""
        check(lib().pw_tri_specialize(self.handle))
        return self

    def group_program(self, G: int) -> np.ndarray:
        """The handle's group program for G = 2 or 4 lanes per mask (host copy)."""
        n = ctypes.c_int32()
        check(lib().pw_tri_group_program(self.handle, int(G), None, 0, ctypes.byref(n)))
        w = np.zeros(n.value, dtype=np.uint32)
        check(lib().pw_tri_group_program(self.handle, int(G), w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                         n.value, ctypes.byref(n)))
        return w

    def program(self) -> np.ndarray:
        """The handle's program words (host copy)."""
        n = ctypes.c_int32()
        check(lib().pw_tri_program(self.handle, None, 0, ctypes.byref(n)))
        w = np.zeros(n.value, dtype=np.uint32)
        check(lib().pw_tri_program(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), n.value,
                                   ctypes.byref(n)))
        return w

    def errors(self) -> int:
        f = ctypes.c_uint32()
        check(lib().pw_tri_errors(self.handle, ctypes.byref(f)))
        return f.value

    def batch(self, masks, codes=None, stream=None):
        """Scheme codes of device masks -> (n,2) int64 device tensor."""
        import torch

        n = masks.numel() * masks.element_size() // mask_bytes(self.d)
        if codes is None:
            codes = torch.empty((n, 2), dtype=torch.int64, device=masks.device)
        check(lib().patchwork_scheme_batch(self.handle, _ptr(masks), n, _ptr(codes), _stream(stream)))
        return codes

    def histogram(self, masks, hist: "Histogram", index_base: int = 0, stream=None):
        n = masks.numel() * masks.element_size() // mask_bytes(self.d)
        check(lib().patchwork_scheme_histogram(self.handle, _ptr(masks), n, int(index_base), hist.handle,
                                               _stream(stream)))

    def codes_histogram(self, masks, hist: "Histogram", codes=None, index_base: int = 0, stream=None):
        """Codes and histogram of the same masks in one pass -> codes."""
        import torch

        n = masks.numel() * masks.element_size() // mask_bytes(self.d)
        if codes is None:
            codes = torch.empty((n, 2), dtype=torch.int64, device=masks.device)
        check(lib().patchwork_scheme_codes_histogram(self.handle, _ptr(masks), n, int(index_base), _ptr(codes),
                                                     hist.handle, _stream(stream)))
        return codes

    def enumerate_range(self, first: int, count: int, hist: "Histogram", fixed_zero_bits: int = 1, stream=None):
        fz = (ctypes.c_uint64 * 2)(fixed_zero_bits & 0xFFFFFFFFFFFFFFFF, fixed_zero_bits >> 64)
        check(lib().patchwork_scheme_enumerate_range(self.handle, int(first), int(count), fz, hist.handle,
                                                     _stream(stream)))

    def sweep_graph(self, first: int, count: int, chunk: int, hist: "Histogram", fixed_zero_bits: int = 1,
                    stream=None):
        """enumerate_range as a chunked sweep captured into a HIP graph
        (kept by the handle and launched again for the same arguments)."""
        fz = (ctypes.c_uint64 * 2)(fixed_zero_bits & 0xFFFFFFFFFFFFFFFF, fixed_zero_bits >> 64)
        check(lib().patchwork_scheme_sweep_graph(self.handle, int(first), int(count), int(chunk), fz, hist.handle,
                                                 _stream(stream)))


def _edges16(edges):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int16).reshape(-1, 4))
    return e, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int16))


def jit_source(d: int, edges) -> str:
    """Source of the kernels specialised to one triangulation."""
    e, p = _edges16(edges)
    n = ctypes.c_int64()
    check(lib().pw_jit_source(d, p, len(e), None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    check(lib().pw_jit_source(d, p, len(e), buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def jit_compile(d: int, edges) -> int:
    """Compile (not load) the specialised kernels; code object bytes."""
    e, p = _edges16(edges)
    n = ctypes.c_int64()
    check(lib().pw_jit_compile(d, p, len(e), ctypes.byref(n)))
    return n.value


def canonical(d: int, edges):
    """S3-canonical member of the triangulation's orbit: (edges (n,4)
    int16, permutation index mapping the input to it, stabiliser order)."""
    e, p = _edges16(edges)
    out = np.zeros_like(e)
    k, st = ctypes.c_int32(), ctypes.c_int32()
    check(lib().pw_tri_canonical(d, p, len(e), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)), ctypes.byref(k),
                                 ctypes.byref(st)))
    return out, k.value, st.value


def point_map(d: int, perm_index: int) -> np.ndarray:
    """Image index of every lattice point under an S3 permutation."""
    out = np.zeros((d + 1) * (d + 2) // 2, dtype=np.int32)
    check(lib().pw_point_map(d, perm_index, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return out


def class_fixed_bits(d: int) -> int:
    """fixed_zero_bits of the (Z/2)^3 class representatives (as an int)."""
    out = (ctypes.c_uint64 * 2)()
    check(lib().pw_class_fixed_bits(d, out))
    return int(out[0]) | (int(out[1]) << 64)


class Histogram:
    """Device histogram code -> (count, witness) (pw_hist_create)."""

    def __init__(self, capacity: int = 4096):
        h = ctypes.c_void_p()
        check(lib().pw_hist_create(int(capacity), ctypes.byref(h)))
        self.handle = h
        self.capacity = int(capacity)

    def close(self):
        if self.handle:
            lib().pw_hist_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        check(lib().pw_hist_reset(self.handle, _stream(stream)))

    def read(self):
        """{code: (count, witness)} sorted by code (synchronises)."""
        cap = self.capacity
        codes = np.zeros((cap, 2), dtype=np.uint64)
        counts = np.zeros(cap, dtype=np.uint64)
        wit = np.zeros(cap, dtype=np.uint64)
        n = ctypes.c_int32()
        u64p = ctypes.POINTER(ctypes.c_uint64)
        check(lib().pw_hist_read(self.handle, codes.ctypes.data_as(u64p), counts.ctypes.data_as(u64p),
                                 wit.ctypes.data_as(u64p), cap, ctypes.byref(n)))
        out = {}
        for k in range(n.value):
            out[int(codes[k, 0]) | (int(codes[k, 1]) << 64)] = (int(counts[k]), int(wit[k]))
        return out


def batch_multi(tris, masks128, offsets, hists=None, codes=None, config=None, stream=None, noalloc=False):
    """Many triangulations (any mix of degrees) in one call: one persistent
    launch per LDS class of degrees, back to back on the stream.

    masks128: device int64 tensor holding two words per mask; triangulation
    t owns masks [offsets[t], offsets[t+1]).  hists: list of Histogram (one
    per triangulation) or None; codes: (n,2) int64 device tensor or None.
    config: (chunk, waves_per_block, blocks_per_cu[, lane_groups]) -- a
    missing lane_groups is DEFAULT_LANE_GROUPS -- or None for the tuned
    shape from the tuning cache (defaults if there is none).  noalloc: use
    patchwork_scheme_batch_multi_noalloc (the library's fixed device array
    instead of buffers it allocates)."""
    n = len(tris)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if len(off) != n + 1:
        raise ValueError("offsets must have len(tris) + 1 entries")
    th = (ctypes.c_void_p * n)(*[t.handle for t in tris])
    hh = (ctypes.c_void_p * n)(*[h.handle for h in hists]) if hists is not None else None
    if config is None:
        from . import tune

        config = tune.lookup_multi([t.d for t in tris])
    if config is not None and len(config) == 3:
        config = (*config, DEFAULT_LANE_GROUPS)
    cfg = MultiConfig(*config) if config is not None else None
    fn = lib().patchwork_scheme_batch_multi_noalloc if noalloc else lib().patchwork_scheme_batch_multi
    check(fn(
        th, n, _ptr(masks128), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        hh, _ptr(codes) if codes is not None else None, ctypes.byref(cfg) if cfg is not None else None,
        _stream(stream)))
    return codes


# ---------------------------------------------------------------- search
# Triangulations on the device: int64 tensors of shape (n, 64), row p =
# neighbour bits of lattice point p (pw_flip_walk and the calls below).

def program_words(d: int) -> int:
    n = lib().pw_program_words(d)
    if n < 0:
        raise PatchworkError(n, "degree out of range")
    return n


def adjacency_from_edges(d: int, edges) -> np.ndarray:
    """Edge list -> 64 adjacency rows (uint64; validated as pw_tri_create)."""
    e, p = _edges16(edges)
    rows = np.zeros(64, dtype=np.uint64)
    check(lib().pw_adjacency_from_edges(d, p, len(e), rows.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return rows


def edges_from_adjacency(d: int, rows) -> np.ndarray:
    """64 adjacency rows -> edge list (n, 4) int16."""
    r = np.ascontiguousarray(np.asarray(rows).view(np.uint64).reshape(64))
    rp = r.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    n = ctypes.c_int32()
    check(lib().pw_edges_from_adjacency(d, rp, None, 0, ctypes.byref(n)))
    out = np.zeros((n.value, 4), dtype=np.int16)
    check(lib().pw_edges_from_adjacency(d, rp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)), n.value,
                                        ctypes.byref(n)))
    return out


def flip_walk(d: int, adj, steps: int, symmetric: bool, seed: int, step0: int = 0, moves=None, stream=None):
    """`steps` random flip moves on every triangulation of adj (in place)."""
    check(lib().pw_flip_walk(d, _ptr(adj), adj.shape[0], int(steps), int(bool(symmetric)), int(seed), int(step0),
                             _ptr(moves) if moves is not None else None, _stream(stream)))


def build_programs(d: int, adj, progs=None, bad=None, stream=None):
    """Diamond programs of every triangulation of adj -> (progs, bad)."""
    import torch

    n = adj.shape[0]
    if progs is None:
        progs = torch.empty((n, program_words(d)), dtype=torch.int32, device=adj.device)
    if bad is None:
        bad = torch.empty(n, dtype=torch.int32, device=adj.device)
    check(lib().pw_build_programs(d, _ptr(adj), n, _ptr(progs), _ptr(bad), _stream(stream)))
    return progs, bad


def scheme_programs(d: int, progs, masks128, codes=None, hist=None, err=None, stream=None):
    """Codes of every (triangulation, witness) pair: progs (n, words),
    masks128 two int64 words per witness -> codes (n * n_w, 2) or None."""
    import torch

    n_tris = progs.shape[0]
    n_w = masks128.numel() // 2
    if err is None:
        err = torch.zeros(1, dtype=torch.int32, device=progs.device)
    check(lib().patchwork_scheme_programs(d, _ptr(progs), n_tris, _ptr(masks128), n_w,
                                          _ptr(codes) if codes is not None else None,
                                          hist.handle if hist is not None else None, _ptr(err), _stream(stream)))
    return codes, err


def tri_objective(d: int, codes, n_tris: int, n_w: int, mode: int = 0, target=(0, 0), known=None, score=None,
                  stream=None):
    """Per-triangulation score over its n_w codes: mode 0 distinct codes,
    mode 1 codes with (p, n) = target, mode 2 distinct codes whose low word
    is not in `known` (sorted int64 device tensor)."""
    import torch

    if score is None:
        score = torch.empty(n_tris, dtype=torch.float32, device=codes.device)
    nk = int(known.numel()) if known is not None else 0
    check(lib().pw_tri_objective(d, _ptr(codes), n_tris, n_w, mode, int(target[0]), int(target[1]),
                                 _ptr(known) if nk else None, nk, _ptr(score), _stream(stream)))
    return score


def anneal_accept(cur, prop, score_cur, score_prop, best, score_best, accept_table, seed: int, step: int,
                  n_accepted, stream=None):
    """Metropolis accept/reject of every chain (pw_anneal_accept)."""
    n = cur.shape[0]
    check(lib().pw_anneal_accept(_ptr(cur), _ptr(prop), _ptr(score_cur), _ptr(score_prop), _ptr(best),
                                 _ptr(score_best), n, _ptr(accept_table), accept_table.numel(), int(seed), int(step),
                                 _ptr(n_accepted), _stream(stream)))
