"""The kernels' evaluation logic, compiled for the CPU, against the oracle.

The per-triangulation evaluator that the library generates (the same source
hipRTC compiles for gfx950) is compiled here with g++ together with the
device header, through tests/host_shim.h, and run lane by lane over one
wave's LDS area.  Every code must equal the oracle's, and a lane may only
write its own bytes of the area (entries, words, parent-table rows).  No GPU
is needed; wave-level parts (histogram, ballots) are not covered here.  The
sweep kernel's evaluator (a snapshot of the fixed-sign part, restored per
batch) is checked the same way, with the snapshot taken from another mask."""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2604_09221_amd import inputs as I
from paper_2604_09221_amd import patchwork as pw

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2604_09221_amd", "csrc")

MAIN = r'''
Dim3E threadIdx{0, 0, 0}, blockIdx{0, 0, 0}, blockDim{64, 1, 1}, gridDim{1, 1, 1};
#include <algorithm>
#include <cstring>
#include <vector>
using C = pw::Cfg<DEG>;
static const size_t kBytes = (size_t)C::LANE_WORDS * 64 * 4;
// the bytes of the wave's area that a lane may write: its entry row (the
// entries, the spare entry and the padding), its words and its
// parent-table bytes
static void own_bytes(int lane, std::vector<unsigned char>& own) {
  memset(own.data(), 0, kBytes);
  for (int k = 0; k < C::LOW_WORDS; ++k)
    for (int b = 0; b < 4; ++b) own[k * 256 + 4 * lane + b] = 1;
  for (int b = 0; b < 4 * C::E_WORDS; ++b) own[lane * 4 * C::E_WORDS + b] = 1;
  for (int x = 0; x < 4 * C::PAR_WORDS; ++x) own[C::PAR_BASE * 256 + x * 64 + lane] = 1;
}
static bool foreign_write(const std::vector<unsigned char>& own, const std::vector<unsigned char>& before,
                          const uint32_t* smem) {
  const unsigned char* cur = (const unsigned char*)smem;
  for (size_t b = 0; b < kBytes; ++b)
    if (!own[b] && cur[b] != before[b]) return true;
  return false;
}
int main(int argc, char** argv) {
  const long n = atol(argv[1]);
  std::vector<uint64_t> in(2 * n), out(2 * n);
  if (fread(in.data(), 8, 2 * n, stdin) != (size_t)(2 * n)) return 3;
  uint32_t* smem = (uint32_t*)aligned_alloc(16, kBytes);
  memset(smem, 0xAB, kBytes);
  std::vector<unsigned char> before(kBytes), own(kBytes);
  long foreign = 0;
  for (long i = 0; i < n; ++i) {
    const int lane = (int)(i % 64);
    typename C::Mask m = (typename C::Mask)in[2 * i];
    if (sizeof(m) == 16) m |= (typename C::Mask)((pw::u128)in[2 * i + 1] << 64);
    uint32_t errs = 0;
#ifdef SNAP
    // the sweep kernel's evaluator: every lane of the wave takes the
    // snapshot of the fixed-sign part from its own mask, which differs
    // from m only in the varying bits 1..9
    typename C::Mask m1 = m ^ (typename C::Mask)((((uint64_t)i * 0x9E3779B97F4A7C15ull) >> 40) & 0x3FEull);
    alignas(16) static uint8_t srow[C::SNAP_BYTES];
    // the wave's lanes build the snapshot row together; here one lane
    // after the other, round by round, until no label goes down (the same
    // fixed point as in lockstep: labels only decrease)
    const std::vector<unsigned char> before_snap((unsigned char*)smem, (unsigned char*)smem + kBytes);
    using S = pw::JitSnap;
    std::vector<S::Links> links;
    for (int j = 0; j < 64; ++j) S::snap_init(srow, j);
    for (int j = 0; j < 64; ++j)
      links.push_back(S::snap_links((uint64_t)((m1 & ~(typename C::Mask)0x7E) | (typename C::Mask)(j << 1)), j));
    for (bool any = true; any;) {
      any = false;
      for (int j = 0; j < 64; ++j) any = S::snap_step(links[j], srow, j) || any;
    }
    if (memcmp(before_snap.data(), smem, kBytes) != 0) ++foreign;  // the label propagation uses its own row only
#ifdef SNAP_PAIRS
    // even d: the per-chunk reduction of the fixed-sign antipodal pairs,
    // one stage after the other, each stage one lane after the other (on
    // the device the stages are separated by wave barriers); a lane may
    // write its own bytes of the area (and the shared snapshot words)
    uint64_t kinds[64];
    for (int stage = 1; stage <= 3; ++stage)
      for (int j = 0; j < 64; ++j) {
        threadIdx.x = j;
        const pw::Lane Lj = pw::lane_memory<DEG>(smem, C::LANE_WORDS);
        own_bytes(j, own);
        memcpy(before.data(), smem, kBytes);
        if (stage == 1) kinds[j] = S::pairs_1(Lj, srow, j);
        if (stage == 2) S::pairs_2(Lj, srow, j);
        if (stage == 3) S::pairs_3(Lj, srow, j, kinds[j]);
        if (foreign_write(own, before, smem)) ++foreign;
      }
#endif
#ifdef SNAP_HITS
    // odd d: the per-chunk reduction of the crossing tests of tree edges
    // between fixed-sign vertices, stage by stage, lane by lane (shared
    // snapshot words only)
    for (int j = 0; j < 64; ++j) S::hits_1(srow, j, (uint64_t)m1);
    for (int j = 0; j < 64; ++j) S::hits_2(srow, j);
    if (memcmp(before_snap.data(), smem, kBytes) != 0) ++foreign;
    {
      // the kept edges, recomputed here: among the crossed tree edges
      // (v, t) between fixed-sign vertices with v not a snapshot root, the
      // first of each unordered pair of snapshot roots
      const uint8_t* row = srow;
      const uint32_t* hx = reinterpret_cast<const uint32_t*>(srow) + C::SNAP_HX;
      std::vector<std::pair<int, int>> seen;
      for (int e = 0; e < S::kNH; ++e) {
        const uint32_t x = pw::kHitEdges[e];
        const int v = (int)(x & 0xFF), t = (int)((x >> 8) & 0xFF);
        const int sv = (int)(((uint64_t)m1 >> ((x >> 16) & 0x7F)) & 1), st = (int)(((uint64_t)m1 >> ((x >> 23) & 0x7F)) & 1);
        const bool crossed = (sv ^ st ^ (int)(x >> 30)) != 0;
        bool keep = false;
        if (row[v] != v && crossed) {
          const std::pair<int, int> key(std::min(row[v], row[t]), std::max(row[v], row[t]));
          keep = std::find(seen.begin(), seen.end(), key) == seen.end();
          if (keep) seen.push_back(key);
        }
        if (keep != (((hx[e / 32] >> (e % 32)) & 1u) != 0)) return 6;
      }
    }
#endif
#endif
    threadIdx.x = lane;
    const pw::Lane L = pw::lane_memory<DEG>(smem, C::LANE_WORDS);
    own_bytes(lane, own);
    memcpy(before.data(), smem, kBytes);
#ifdef SNAP
    const auto fl = pw::JitSnap{}.flags(m1, srow);
    const pw::u128 code = pw::JitSnap{}.batch(m, L, srow, fl, errs);
#else
    const pw::u128 code = pw::JitEval{}(m, L, errs);
#endif
    out[2 * i] = errs ? 0 : (uint64_t)code;
    out[2 * i + 1] = errs ? 0 : (uint64_t)(code >> 64);
    if (foreign_write(own, before, smem)) ++foreign;
  }
  fwrite(out.data(), 8, 2 * n, stdout);
  free(smem);
  return foreign ? 4 : 0;
}
'''


def _compile(tmp_path, d, edges, snap):
    src = pw.jit_source(d, edges)
    src = src[:src.index('extern "C"')]          # the evaluators; the kernels need a GPU
    path = tmp_path / f"emu_d{d}.cpp"
    defs = ("#define SNAP 1\n" if snap else "") + ("#define SNAP_PAIRS 1\n" if snap and d % 2 == 0 else "") + \
        ("#define SNAP_HITS 1\n" if snap and d % 2 == 1 else "")
    path.write_text(defs + '#include "host_shim.h"\n' + src + MAIN.replace("DEG", str(d)))
    exe = tmp_path / f"emu_d{d}"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-w", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-I", HERE, "-I", CSRC, "-o", str(exe), str(path)])
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("d,noise,seed,n,snap", [(4, None, 0, 3000, False), (5, 1.0, 2, 2000, False),
                                                 (6, 1.0, 3, 2000, False), (7, None, 0, 3000, False),
                                                 (7, 1.0, 4, 2000, False), (9, None, 0, 600, False),
                                                 (6, 1.0, 5, 2000, True), (5, 1.0, 2, 2000, True), (7, None, 0, 3000, True),
                                                 (7, 1.0, 6, 2000, True), (8, None, 0, 600, True),
                                                 (9, None, 0, 600, True)])
def test_evaluator_on_host_matches_oracle(tmp_path, d, noise, seed, n, snap):
    edges = I.standard_triangulation(d) if noise is None else I.lift_triangulation(d, seed, noise=noise)
    _check(tmp_path, d, edges, seed, n, snap)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("name", ["bow_tie", "rank016"])
def test_sweep_evaluator_on_fig2_triangulations(tmp_path, name):
    """The sweep kernel's evaluator on two of the degree-8 triangulations
    of Fig. 2.  On bow_tie the fixed-sign pairs close an odd cycle in every
    chunk (a mark left to each batch); on rank016 more of the pair sets are
    out of the varying vertices' reach (merged into the snapshot)."""
    edges = np.loadtxt(os.path.join(HERE, "golden", f"fig2_{name}.edges"), dtype=np.int32)
    _check(tmp_path, 8, edges, 9, 400, True)


def _check(tmp_path, d, edges, seed, n, snap):
    exe = _compile(tmp_path, d, edges, snap)
    masks = np.ascontiguousarray(I.random_masks(d, seed + 11, n).astype(np.uint64))
    # first rows: the Harnack distribution (the most regions), all '+', all
    # '-' except sigma(0,0), and every single flip of the Harnack mask
    nA = I.n_points(d)
    h = I.harnack_mask(d)
    special = [h, 0, ((1 << nA) - 1) & ~1] + [h ^ (1 << k) for k in range(1, nA)]
    for i, x in enumerate(special[:n]):
        masks[i, 0] = x & ((1 << 64) - 1)
        masks[i, 1] = x >> 64
    run = subprocess.run([str(exe), str(n)], input=masks.tobytes(), capture_output=True)
    assert run.returncode != 4, "a lane wrote outside its own LDS bytes"
    assert run.returncode != 6, "the sweep kernel kept the wrong crossing tests of a chunk"
    assert run.returncode == 0, run.stderr.decode()[-2000:]
    got = np.frombuffer(run.stdout, dtype=np.uint64).reshape(n, 2)
    want = oracle.scheme_many(d, edges, masks, threads=4)
    assert np.array_equal(got, want)
