"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle,
bit-exact on every scheme code, histogram count and witness.

Sizes: small enough for the oracle to finish in seconds while spanning many
waves and a ragged tail; full workload sizes are checked on sampled outputs
and on properties that hold at any size (sums, (Z/2)^2 orbit divisibility,
witness validity, the bound of 121 schemes in degree 7)."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from paper_2604_09221_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def pw():
    from paper_2604_09221_amd import patchwork

    assert torch.cuda.is_available()
    patchwork.lib()
    return patchwork


def fig2_edges(name):
    return np.loadtxt(os.path.join(GOLD, f"fig2_{name}.edges"), dtype=np.int32)


def gpu_codes(pw, d, E, masks2):
    tri = pw.Triangulation(d, E)
    out = tri.batch(pw.mask_tensor(masks2, d))
    torch.cuda.synchronize()
    assert tri.errors() == 0
    return out.cpu().numpy().view(np.uint64)


def oracle_hist(codes2, index_of=None):
    """{code: (count, smallest index)} of an (n,2) code array."""
    codes2 = np.ascontiguousarray(codes2, dtype=np.uint64)
    idx = np.arange(len(codes2), dtype=np.uint64) if index_of is None else np.asarray(index_of, dtype=np.uint64)
    keys, first, inv, counts = np.unique(codes2, axis=0, return_index=True, return_inverse=True,
                                         return_counts=True)
    wmin = np.full(len(keys), np.iinfo(np.uint64).max, dtype=np.uint64)
    np.minimum.at(wmin, inv.reshape(-1), idx)
    return {int(lo) | (int(hi) << 64): (int(c), int(w)) for (lo, hi), c, w in zip(keys, counts, wmin)}


def enum_masks(first, count, fixed=1, nA=64):
    free = [b for b in range(nA) if not (fixed >> b) & 1]
    out = np.zeros((count, 2), dtype=np.uint64)
    idx = np.arange(first, first + count, dtype=np.uint64)
    lo = np.zeros(count, dtype=np.uint64)
    hi = np.zeros(count, dtype=np.uint64)
    for k, b in enumerate(free[:64]):
        bit = (idx >> np.uint64(k)) & np.uint64(1)
        if b < 64:
            lo |= bit << np.uint64(b)
        else:
            hi |= bit << np.uint64(b - 64)
    out[:, 0], out[:, 1] = lo, hi
    return out


# ------------------------------------------------------------------ d = 4

@pytest.mark.parametrize("which", ["std", "lift1", "lift2", "lift3"])
def test_d4_exhaustive_codes_and_histogram(pw, which):
    d = 4
    E = I.standard_triangulation(d) if which == "std" else I.lift_triangulation(d, int(which[-1]), noise=1.0)
    masks = enum_masks(0, 1 << 14, nA=15)
    want = oracle.scheme_many(d, E, masks, threads=THREADS)
    got = gpu_codes(pw, d, E, masks)
    assert np.array_equal(got, want)
    tri = pw.Triangulation(d, E)
    hist = pw.Histogram(256)
    tri.enumerate_range(0, 1 << 14, hist)
    h = hist.read()
    assert h == oracle_hist(want)
    assert sum(c for c, _ in h.values()) == 1 << 14
    assert all(c % 4 == 0 for c, _ in h.values())   # free (Z/2)^2 orbits of the sign action
    assert tri.errors() == 0


# ---------------------------------------------------------------- d = 1..3

def test_small_degrees_all_masks(pw):
    for d in (1, 2, 3):
        Es = [I.standard_triangulation(d)] + ([I.lift_triangulation(d, s, noise=1.0) for s in range(3)] if d > 1 else [])
        for E in Es:
            n = 1 << I.n_points(d)
            masks = np.zeros((n, 2), dtype=np.uint64)
            masks[:, 0] = np.arange(n, dtype=np.uint64)       # bit 0 set too
            assert np.array_equal(gpu_codes(pw, d, E, masks), oracle.scheme_many(d, E, masks))


# ------------------------------------------------------------------ d = 6

def test_d6_varied_triangulations_ragged(pw):
    d = 6
    for seed in range(6):
        E = I.lift_triangulation(d, seed, noise=1.0) if seed else I.lift_triangulation(d, 0, noise=0.05)
        n = (1 << 15) + 37 * seed + 1
        masks = I.random_masks(d, seed, n)
        assert np.array_equal(gpu_codes(pw, d, E, masks), oracle.scheme_many(d, E, masks, threads=THREADS))


def test_d6_full_size_sampled(pw):
    """64 triangulations (lift seeds 0..63, literal and varied) x 2^20 masks,
    as the workload runs; 256 sampled outputs per slot against the oracle,
    plus the histogram API on every slot against the codes."""
    d = 6
    rng = np.random.default_rng(6)
    for noise in (0.05, 1.0):
        for seed in range(0, 64, 9 if noise == 1.0 else 21):
            E = I.lift_triangulation(d, seed, noise=noise)
            masks = I.random_masks(d, seed, 1 << 20)
            mt = pw.mask_tensor(masks, d)
            tri = pw.Triangulation(d, E)
            codes = tri.batch(mt)
            hist = pw.Histogram(256)
            tri.histogram(mt, hist, index_base=1000)
            torch.cuda.synchronize()
            got = codes.cpu().numpy().view(np.uint64)
            pick = rng.choice(len(masks), 256, replace=False)
            assert np.array_equal(got[pick], oracle.scheme_many(d, E, masks[pick], threads=THREADS))
            h = hist.read()
            assert h == oracle_hist(got, index_of=np.arange(1000, 1000 + len(masks)))
            assert len(h) <= 55
            assert tri.errors() == 0


# ------------------------------------------------------------------ d = 7

def test_d7_subsample_codes(pw):
    """SplitMix64 stream 7: idx = low 35 bits, mask = idx << 1."""
    d = 7
    E = I.lift_triangulation(d, 7, noise=0.05)
    n = (1 << 20) + 13
    idx = I.subsample_indices(7, n, 35)
    masks = np.zeros((n, 2), dtype=np.uint64)
    masks[:, 0] = idx << np.uint64(1)
    assert np.array_equal(gpu_codes(pw, d, E, masks), oracle.scheme_many(d, E, masks, threads=THREADS))


@pytest.mark.parametrize("first,count", [(0, 1 << 20), (123457, 100003), (2**35 - 5000, 5000)])
def test_d7_enumerate_range_histogram(pw, first, count):
    d = 7
    E = I.standard_triangulation(d)
    masks = enum_masks(first, count, nA=36)
    want = oracle.scheme_many(d, E, masks, threads=THREADS)
    tri = pw.Triangulation(d, E)
    hist = pw.Histogram(512)
    tri.enumerate_range(first, count, hist)
    assert hist.read() == oracle_hist(want, index_of=np.arange(first, first + count, dtype=np.uint64))
    assert tri.errors() == 0


def test_d7_large_range_properties(pw):
    """2^30 enumerated masks: counts sum to the range, at most 121 schemes
    (Sec. 1), and every witness reproduces its code on the oracle."""
    d = 7
    E = I.standard_triangulation(d)
    tri = pw.Triangulation(d, E)
    hist = pw.Histogram(512)
    tri.enumerate_range(0, 1 << 30, hist)
    h = hist.read()
    assert sum(c for c, _ in h.values()) == 1 << 30
    assert len(h) <= 121
    wit = np.array([w for _, w in h.values()], dtype=np.uint64)
    masks = np.zeros((len(wit), 2), dtype=np.uint64)
    masks[:, 0] = wit << np.uint64(1)
    want = oracle.scheme_many(d, E, masks)
    assert [int(lo) | (int(hi) << 64) for lo, hi in want] == list(h.keys())
    assert tri.errors() == 0


@pytest.mark.parametrize("d", [5, 6])
def test_whole_sweeps_specialised_equal_generic(pw, d):
    """All 2^(nA - 1) masks of a varied triangulation (sigma(0,0) = +): the
    specialised sweep kernel (shared snapshot, per-chunk reduction of the
    crossing tests at odd d and of the antipodal pairs at even d) gives the
    histogram of the generic kernel, counts and witnesses; the counts sum to
    the sweep and are divisible by 4 (sigma -> sigma + b i + c j, (b, c) !=
    (0, 0), keeps sigma(0,0) and the scheme and has no fixed point: a free
    (Z/2)^2 action on a whole sweep); every witness's code is the oracle's."""
    E = I.lift_triangulation(d, 4, noise=1.0)
    total = 1 << (I.n_points(d) - 1)
    spec = pw.Triangulation(d, E).specialize()
    gen = pw.Triangulation(d, E)
    h1, h2 = pw.Histogram(512), pw.Histogram(512)
    spec.enumerate_range(0, total, h1)
    gen.enumerate_range(0, total, h2)
    a, b = h1.read(), h2.read()
    assert a == b
    assert sum(c for c, _ in a.values()) == total
    assert all(c % 4 == 0 for c, _ in a.values())
    wit = np.array([w for _, w in a.values()], dtype=np.uint64)
    masks = np.zeros((len(wit), 2), dtype=np.uint64)
    masks[:, 0] = wit << np.uint64(1)
    want = oracle.scheme_many(d, E, masks)
    assert [int(lo) | (int(hi) << 64) for lo, hi in want] == list(a.keys())
    assert spec.errors() == 0 and gen.errors() == 0


# ------------------------------------------------------------------ d = 8

@pytest.mark.parametrize("name", ["bow_tie", "rank016", "rank015"])
def test_d8_figure2_triangulations(pw, name):
    d = 8
    E = fig2_edges(name)
    masks = I.random_masks(d, 8, (1 << 17) + 5)
    assert np.array_equal(gpu_codes(pw, d, E, masks), oracle.scheme_many(d, E, masks, threads=THREADS))


# -------------------------------------------------------------- d = 9..12

@pytest.mark.parametrize("d", [5, 9, 10, 11, 12])
def test_wide_masks_and_large_degrees(pw, d):
    for seed in (1, 2):
        E = I.lift_triangulation(d, seed, noise=1.0)
        masks = I.random_masks(d, seed, 4096 + 3 * seed)
        masks[:, 0] |= np.uint64(seed & 1)                 # bit 0 may be set
        assert np.array_equal(gpu_codes(pw, d, E, masks), oracle.scheme_many(d, E, masks, threads=THREADS))
    # the Harnack distribution: an M-curve on every triangulation
    E = I.standard_triangulation(d)
    m = I.harnack_mask(d)
    masks = np.array([[m & (2**64 - 1), m >> 64]], dtype=np.uint64)
    assert np.array_equal(gpu_codes(pw, d, E, masks), oracle.scheme_many(d, E, masks))


@pytest.mark.parametrize("d", [10, 11, 12])
def test_large_degrees_histogram_and_enumeration(pw, d):
    """Degrees 10..12 evaluate one mask with a group of four lanes (one
    reflected quadrant each): histograms with an index base, the fused
    codes + histogram call and enumerated index ranges, bit-exact (codes,
    counts and witnesses) against the oracle."""
    E = I.lift_triangulation(d, 3, noise=1.0)
    tri = pw.Triangulation(d, E)
    nA = I.n_points(d)
    masks = I.random_masks(d, 70 + d, 5003)
    h = I.harnack_mask(d)
    flips = [h] + [h ^ (1 << b) for b in range(1, nA, 5)]       # many regions (the full phase-4 tables)
    for k, x in enumerate(flips):
        masks[k, 0], masks[k, 1] = x & (2**64 - 1), x >> 64
    want = oracle.scheme_many(d, E, masks, threads=THREADS)
    mt = pw.mask_tensor(masks, d)
    hist = pw.Histogram(8192)
    tri.histogram(mt, hist, index_base=1000)
    assert hist.read() == oracle_hist(want, index_of=np.arange(1000, 1000 + len(masks), dtype=np.uint64))
    hist2 = pw.Histogram(8192)
    codes = torch.zeros((len(masks), 2), dtype=torch.int64, device="cuda")
    tri.codes_histogram(mt, hist2, codes)
    assert np.array_equal(codes.cpu().numpy().view(np.uint64), want)
    assert hist2.read() == oracle_hist(want)
    for first, n in [(0, 4099), ((1 << 40) + 12345, 3001), ((1 << 64) - 2000, 1999)]:
        he = pw.Histogram(8192)
        tri.enumerate_range(first, n, he)
        wm = oracle.scheme_many(d, E, enum_masks(first, n, fixed=1, nA=nA), threads=THREADS)
        assert he.read() == oracle_hist(wm, index_of=np.arange(first, first + n, dtype=np.uint64))
    assert tri.errors() == 0


# -------------------------------------------------------------- edge cases

def test_edge_cases(pw):
    d = 7
    E = I.standard_triangulation(d)
    tri = pw.Triangulation(d, E)
    empty = torch.empty(0, dtype=torch.int64, device="cuda")
    out = torch.empty((0, 2), dtype=torch.int64, device="cuda")
    tri.batch(empty, out)                                   # n = 0 is a no-op
    for n in (1, 63, 64, 65, 257):
        masks = I.random_masks(d, n, n)
        assert np.array_equal(gpu_codes(pw, d, E, masks), oracle.scheme_many(d, E, masks))
    assert pw.lib().patchwork_scheme_batch(tri.handle, None, -1, None, None) == pw.PW_ERR_ARG
    hist = pw.Histogram(64)
    with pytest.raises(pw.PatchworkError) as e:
        tri.enumerate_range(2**35 - 10, 11, hist)
    assert e.value.status == pw.PW_ERR_RANGE
    tri.enumerate_range(0, 0, hist)                        # empty range
    small = pw.Histogram(16)
    tri.enumerate_range(0, 1 << 20, small)                  # > 16 schemes
    with pytest.raises(pw.PatchworkError) as e:
        small.read()
    assert e.value.status == pw.PW_ERR_HIST_FULL
    # class representatives: (0,0), (1,0), (0,1) fixed
    fixed = (1 << 0) | (1 << 1) | (1 << (d + 1))
    reps = pw.Histogram(512)
    tri.enumerate_range(0, 1 << 20, reps, fixed_zero_bits=fixed)
    masks = enum_masks(0, 1 << 20, fixed=fixed, nA=36)
    want = oracle.scheme_many(d, E, masks, threads=THREADS)
    assert reps.read() == oracle_hist(want)
    assert tri.errors() == 0


# ------------------------------------------------- graph-captured chunked sweep

def test_sweep_graph_replays_match_eager(pw):
    """patchwork_scheme_sweep_graph: a range swept in chunks through a HIP
    graph gives the eager histogram; the kept graph launched again adds the
    same counts (three launches, with eager work and synchronisation in
    between, each checked), and new arguments capture a new graph."""
    for d, spec in ((7, True), (6, False)):
        E = I.standard_triangulation(d)
        tri = pw.Triangulation(d, E)
        if spec:
            tri.specialize()
        first, n, chunk = 777, (1 << 18) + 4321, 1 << 15
        h_eager = pw.Histogram(512)
        tri.enumerate_range(first, n, h_eager)
        want = h_eager.read()
        ref = oracle_hist(oracle.scheme_many(d, E, enum_masks(first, n, nA=I.n_points(d)), threads=THREADS),
                          index_of=np.arange(first, first + n, dtype=np.uint64))
        assert want == ref
        h = pw.Histogram(512)
        for rep in range(1, 4):
            tri.sweep_graph(first, n, chunk, h)
            torch.cuda.synchronize()
            got = h.read()
            assert got == {c: (k * rep, w) for c, (k, w) in want.items()}
            tri.enumerate_range(0, 1000, pw.Histogram(64))     # eager work between the launches
            torch.cuda.synchronize()
        h2 = pw.Histogram(512)
        tri.sweep_graph(first + 5, 2 * chunk + 1, chunk, h2)   # other arguments: a new capture
        torch.cuda.synchronize()
        h3 = pw.Histogram(512)
        tri.enumerate_range(first + 5, 2 * chunk + 1, h3)
        assert h2.read() == h3.read()
        with pytest.raises(RuntimeError):
            tri.sweep_graph(first, n, 0, h)
        assert tri.errors() == 0


# ------------------------------------------------- specialised kernels (hipRTC)

def test_class_representative_sweep(pw):
    """The Fig. 2 sweep's enumeration (d = 8, sigma fixed at (0,0), (1,1),
    (2,1)): histograms of index ranges -- chunk-aligned, ragged and near the
    end of the 2^42 classes -- bit-exact against the oracle."""
    import bench

    fz = bench.fig2_fixed_bits(8)
    for name in ("rank016", "bow_tie"):
        E = fig2_edges(name)
        tri = pw.Triangulation(8, E).specialize()
        for first, n in [(0, 1 << 15), (777, 20001), ((1 << 42) - 3000, 3000)]:
            h = pw.Histogram(1024)
            tri.enumerate_range(first, n, h, fixed_zero_bits=fz)
            want = oracle.scheme_many(8, E, enum_masks(first, n, fixed=fz, nA=45), threads=THREADS)
            assert h.read() == oracle_hist(want, index_of=np.arange(first, first + n, dtype=np.uint64))
        assert tri.errors() == 0


def test_specialized_kernels_match_oracle(pw):
    """Kernels generated for one triangulation: codes, histograms and
    witnesses bit-exact against the oracle (and hence the generic path)."""
    cases = [(4, I.lift_triangulation(4, 2, noise=1.0), 1 << 14),
             (6, I.lift_triangulation(6, 3, noise=1.0), 1 << 15),
             (7, I.standard_triangulation(7), 1 << 18),
             (8, fig2_edges("rank016"), 1 << 16)]
    for d, E, n in cases:
        tri = pw.Triangulation(d, E).specialize()
        masks = I.random_masks(d, d, n + 7)
        out = tri.batch(pw.mask_tensor(masks, d))
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint64), oracle.scheme_many(d, E, masks, threads=THREADS))
        hist = pw.Histogram(1024)
        first = min(1000, (1 << (I.n_points(d) - 1)) - n)
        tri.enumerate_range(first, n, hist)
        emasks = enum_masks(first, n, nA=I.n_points(d))
        want = oracle.scheme_many(d, E, emasks, threads=THREADS)
        assert hist.read() == oracle_hist(want, index_of=np.arange(first, first + n, dtype=np.uint64))
        h2 = pw.Histogram(1024)
        tri.histogram(pw.mask_tensor(masks, d), h2, index_base=5)
        assert h2.read() == oracle_hist(oracle.scheme_many(d, E, masks, threads=THREADS),
                                        index_of=np.arange(5, 5 + len(masks), dtype=np.uint64))
        if d == 7:  # the sweep kernel's last, partial chunk
            h3 = pw.Histogram(1024)
            last = (1 << 35) - 5000
            tri.enumerate_range(last, 5000, h3)
            want3 = oracle.scheme_many(d, E, enum_masks(last, 5000, nA=I.n_points(d)), threads=THREADS)
            assert h3.read() == oracle_hist(want3, index_of=np.arange(last, last + 5000, dtype=np.uint64))
        assert tri.errors() == 0


# ------------------------------------- the timed sweep kernel over its whole range

def _chunks_across_range(rng, n_free, n_aligned, n_ragged, chunk=512):
    """(first, count) pairs: n_aligned whole 512-mask chunks at random
    positions of [0, 2^n_free) (so the fixed-sign pattern of every snapshot
    -- index bits 9 and up -- takes random values), then n_ragged ranges of
    random start and length up to three chunks (partial chunks at both
    ends)."""
    top = 1 << n_free
    out = []
    for _ in range(n_aligned):
        out.append((int(rng.integers(0, top // chunk)) * chunk, chunk))
    for _ in range(n_ragged):
        n = int(rng.integers(1, 3 * chunk))
        out.append((int(rng.integers(0, top - n)), n))
    return out


@pytest.mark.parametrize("d", [7, 6, 9, 5])
def test_d7_sweep_kernel_mid_range(pw, d):
    """The specialised sweep kernel (shared snapshot per 512 masks) on 256
    whole chunks spread over the 2^(nA - 1) indices and 64 ragged ranges:
    histogram counts and witnesses of every range against the oracle.  d = 7
    is the timed sweep; d = 6 (a varied triangulation) covers the even-degree
    reduction of the fixed-sign antipodal pairs with u8 entries that hold
    the parity bit; d = 9 and 5 (varied) the other odd degrees with the
    per-chunk reduction of the crossing tests."""
    E = I.standard_triangulation(d) if d == 7 else I.lift_triangulation(d, 5, noise=1.0)
    tri = pw.Triangulation(d, E).specialize()
    rng = np.random.default_rng(735 + d)
    nA = I.n_points(d)
    ranges = _chunks_across_range(rng, nA - 1, 256, 64)
    hist = pw.Histogram(512)
    allm = np.concatenate([enum_masks(a, n, nA=nA) for a, n in ranges])
    want = oracle.scheme_many(d, E, allm, threads=THREADS)
    pos = 0
    for a, n in ranges:
        hist.reset()
        tri.enumerate_range(a, n, hist)
        assert hist.read() == oracle_hist(want[pos:pos + n], index_of=np.arange(a, a + n, dtype=np.uint64)), (a, n)
        pos += n
    assert tri.errors() == 0


def test_d8_class_sweep_kernel_mid_range(pw):
    """The even-degree sweep kernel on the Fig. 2 class-representative
    enumeration (sigma fixed at (0,0), (1,1), (2,1)): 128 whole chunks
    spread over the 2^42 classes and 32 ragged ranges, per range against
    the oracle."""
    import bench

    fz = bench.fig2_fixed_bits(8)
    rng = np.random.default_rng(842)
    for name in ("rank015", "bow_tie", "rank016"):
        E = fig2_edges(name)
        tri = pw.Triangulation(8, E).specialize()
        ranges = _chunks_across_range(rng, 42, 128, 32)
        allm = np.concatenate([enum_masks(a, n, fixed=fz, nA=45) for a, n in ranges])
        want = oracle.scheme_many(8, E, allm, threads=THREADS)
        hist = pw.Histogram(1024)
        pos = 0
        for a, n in ranges:
            hist.reset()
            tri.enumerate_range(a, n, hist, fixed_zero_bits=fz)
            assert hist.read() == oracle_hist(want[pos:pos + n], index_of=np.arange(a, a + n, dtype=np.uint64)), \
                (name, a, n)
            pos += n
        assert tri.errors() == 0


def test_sweep_graph_new_histogram_after_destroy(pw):
    """A histogram destroyed and created again (the allocator may hand out
    the same address) gets a new capture, not the kept graph of the old
    one: same arguments, fresh histogram, result equal to the eager one."""
    d = 6
    E = I.standard_triangulation(d)
    tri = pw.Triangulation(d, E)
    first, n, chunk = 99, (1 << 16) + 5, 1 << 14
    h_eager = pw.Histogram(256)
    tri.enumerate_range(first, n, h_eager)
    want = h_eager.read()
    for _ in range(3):
        h = pw.Histogram(256)
        tri.sweep_graph(first, n, chunk, h)
        torch.cuda.synchronize()
        assert h.read() == want
        h.close()
    assert tri.errors() == 0


# ------------------------------------------------- codes and histogram in one pass

@pytest.mark.parametrize("spec", [False, True])
def test_codes_histogram_fused(pw, spec):
    """patchwork_scheme_codes_histogram: the codes equal the oracle's and the
    histogram (counts, witnesses) equals the one of those codes, for ragged
    sizes at d = 4, 6 (varied lifts) and 8; a misaligned code buffer is an
    argument error."""
    for d, seed, n in ((4, 1, (1 << 14) - 3), (6, 5, (1 << 16) + 77), (8, 2, 20001)):
        E = I.lift_triangulation(d, seed, noise=1.0)
        tri = pw.Triangulation(d, E)
        if spec:
            tri.specialize()
        masks = I.random_masks(d, 40 + seed, n)
        mt = pw.mask_tensor(masks, d)
        hist = pw.Histogram(1024)
        codes = tri.codes_histogram(mt, hist, index_base=7)
        torch.cuda.synchronize()
        got = codes.cpu().numpy().view(np.uint64)
        want = oracle.scheme_many(d, E, masks, threads=THREADS)
        assert np.array_equal(got, want)
        assert hist.read() == oracle_hist(want, index_of=np.arange(7, 7 + n, dtype=np.uint64))
        assert tri.errors() == 0
    buf = torch.empty((n + 1) * 2, dtype=torch.int64, device="cuda")
    mis = buf[1:2 * n + 1]                                   # 8 bytes off a 16-byte boundary
    with pytest.raises(pw.PatchworkError) as e:
        tri.codes_histogram(mt, hist, codes=mis)
    assert e.value.status == pw.PW_ERR_ARG
    with pytest.raises(pw.PatchworkError) as e:
        tri.batch(mt, mis)
    assert e.value.status == pw.PW_ERR_ARG
