"""The lane-group evaluator of the batched launch, compiled for the CPU,
against the oracle.

pw_group.h (G = 2 or 4 lanes per mask, one reflected block of the diamond
per lane) is compiled with g++ through tests/host_shim.h together with the
host builder of the group programs (tri.cpp), and one group is run the way
the wave runs it: every lane's phase 1 on its own block, phase 2 once (the
lanes of a group run it in lockstep on the same entries with the same
values), every lane's phase 3a, then phase 3b vertex by vertex -- all lanes'
root tests, the group's ballot prefix, all lanes' id writes, then all
lanes' lookups -- and finish() once.  Every code must equal the oracle's,
the group may write only its own part of the wave's area (its entries,
its words of the region tables, its bytes of the parent rows), and the
sanitizers watch every access.  The area starts as 0xAB bytes, so a walk
from an entry never written would go to index 0x1AB, outside the group's
entries.  No GPU is needed."""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2604_09221_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2604_09221_amd", "csrc")

MAIN = r'''
#include "pw_group.h"
#include <cstring>
#include <vector>
Dim3E threadIdx{0, 0, 0}, blockIdx{0, 0, 0}, blockDim{64, 1, 1}, gridDim{1, 1, 1};
using GE = pw::GroupEval<DEG, GRP, RCAP_>;
using GC = GE::GC;
using C = GE::C;
int main(int argc, char** argv) {
  const long n = atol(argv[1]);
  const int n_edges = atoi(argv[2]);
  std::vector<int16_t> edges(4 * n_edges);
  if (fread(edges.data(), 2, 4 * n_edges, stdin) != (size_t)(4 * n_edges)) return 3;
  std::vector<uint64_t> in(2 * n), out(2 * n);
  if (fread(in.data(), 8, 2 * n, stdin) != (size_t)(2 * n)) return 3;
  static pw::HostProgram full;
  char msg[256];
  if (pw::build_program(DEG, edges.data(), n_edges, &full, msg, sizeof msg) != 0) { fprintf(stderr, "%s\n", msg); return 5; }
  std::vector<uint32_t> prog(pw::group_program_words(DEG, GRP));
  if (pw::build_group_program(full, GRP, prog.data(), msg, sizeof msg) != 0) { fprintf(stderr, "%s\n", msg); return 5; }
  const size_t kBytes = (size_t)GC::WAVE_DW * 4;
  uint32_t* wave = (uint32_t*)aligned_alloc(16, (kBytes + 15) / 16 * 16);
  std::vector<unsigned char> before(kBytes), own(kBytes);
  long foreign = 0;
  for (long i = 0; i < n; ++i) {
    const int g = (int)(i % GC::NG);  // the group's place in the wave
    typename C::Mask m = (typename C::Mask)in[2 * i];
    if (sizeof(m) == 16) m |= (typename C::Mask)((pw::u128)in[2 * i + 1] << 64);
    memset(wave, 0xAB, kBytes);
    // the group's bytes
    memset(own.data(), 0, kBytes);
    for (size_t b = 0; b < 4 * (size_t)GC::GROUP_DW; ++b) own[4 * (size_t)g * GC::GROUP_DW + b] = 1;
    for (int k = 0; k < C::TAIL_WORDS; ++k)
      for (int b = 0; b < 4; ++b) own[4 * ((size_t)k * GC::NG + g) + b] = 1;
    for (int x = 0; x <= C::RMAX; ++x) own[4 * (size_t)GC::LOW_DW + (size_t)x * GC::NG + g] = 1;
    memcpy(before.data(), wave, kBytes);
    GE::Mem M[GRP];
    for (int q = 0; q < GRP; ++q) M[q] = GE::memory(wave, g * GRP + q);
    for (int q = 0; q < GRP; ++q) GE::phase1(prog.data(), m ^ GE::flip(q), M[q], q);
    GE::phase2(prog.data(), M[0]);
    for (int q = 0; q < GRP; ++q) GE::phase3a(M[q], q);
    int nR = 0;
    typename C::Adj roots = 0;
    for (int v = 0; v < GC::NB; ++v) {
      bool is_root[GRP];
      uint32_t ev[GRP];
      int cid[GRP];
      int cnt = 0;
      for (int q = 0; q < GRP; ++q) is_root[q] = GE::p3_is_root(M[q], v, q, ev[q]);
      for (int q = 0; q < GRP; ++q) {
        const int id = nR + cnt;  // the ballot prefix: roots of lower lanes at this vertex
        cid[q] = id < C::RMAX ? id : C::RMAX;
        cnt += is_root[q] ? 1 : 0;
      }
      nR += cnt;
      for (int q = 0; q < GRP; ++q) GE::p3_write(M[q], v, is_root[q], cid[q]);
      for (int q = 0; q < GRP; ++q) GE::p3_link(prog.data(), m ^ GE::flip(q), M[q], v, q, is_root[q], ev[q], cid[q], roots);
    }
    uint32_t errs = 0;
    const pw::u128 code = GE::E::finish(M[0].view, nR, roots, errs);
    out[2 * i] = errs ? 0 : (uint64_t)code;
    out[2 * i + 1] = errs ? ((errs & pw::kErrOverflow) ? 1 : 0) : (uint64_t)(code >> 64);
    const unsigned char* cur = (const unsigned char*)wave;
    for (size_t b = 0; b < kBytes; ++b)
      if (!own[b] && cur[b] != before[b]) { ++foreign; break; }
  }
  fwrite(out.data(), 8, 2 * n, stdout);
  free(wave);
  return foreign ? 4 : 0;
}
'''


def _compile(tmp_path, d, G, rcap):
    path = tmp_path / f"group_d{d}_g{G}_r{rcap}.cpp"
    # (pw_internal.h first, without the shim: the host builder's declarations)
    path.write_text('#include "pw_internal.h"\n#include "host_shim.h"\n' +
                    MAIN.replace("DEG", str(d)).replace("GRP", str(G)).replace("RCAP_", str(rcap)))
    exe = tmp_path / f"group_d{d}_g{G}_r{rcap}"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-w", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-I", HERE, "-I", CSRC, "-o", str(exe), str(path),
                           os.path.join(CSRC, "tri.cpp")])
    return exe


def _masks(d, seed, n):
    masks = np.ascontiguousarray(I.random_masks(d, seed + 11, n).astype(np.uint64))
    # first rows: the Harnack distribution (the most regions), all '+', all
    # '-' except sigma(0,0), and single flips of the Harnack mask
    nA = I.n_points(d)
    h = I.harnack_mask(d)
    special = [h, 0, ((1 << nA) - 1) & ~1] + [h ^ (1 << k) for k in range(1, nA, 3)]
    for i, x in enumerate(special[:n]):
        masks[i, 0] = x & ((1 << 64) - 1)
        masks[i, 1] = x >> 64
    return masks


def _run(exe, edges, masks):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int16).reshape(-1, 4))
    run = subprocess.run([str(exe), str(len(masks)), str(len(e))], input=e.tobytes() + masks.tobytes(),
                         capture_output=True)
    assert run.returncode != 4, "a group wrote outside its own part of the wave's area"
    assert run.returncode == 0, run.stderr.decode()[-2000:]
    return np.frombuffer(run.stdout, dtype=np.uint64).reshape(len(masks), 2)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("d,G,noise,seed,n", [(8, 4, None, 0, 400), (8, 2, 1.0, 1, 400), (9, 4, 1.0, 2, 300),
                                              (9, 2, None, 0, 300), (10, 4, 1.0, 3, 200), (10, 2, 1.0, 4, 200),
                                              (11, 4, None, 0, 150), (11, 2, 1.0, 5, 150), (12, 4, 1.0, 6, 120),
                                              (12, 2, None, 0, 120)])
def test_group_evaluator_matches_oracle(tmp_path, d, G, noise, seed, n):
    edges = I.standard_triangulation(d) if noise is None else I.lift_triangulation(d, seed, noise=noise)
    exe = _compile(tmp_path, d, G, 0)
    masks = _masks(d, seed, n)
    got = _run(exe, edges, masks)
    want = oracle.scheme_many(d, edges, masks, threads=4)
    assert np.array_equal(got, want)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("d,G", [(12, 4), (10, 2)])
def test_group_evaluator_capped_tables(tmp_path, d, G):
    """With phase-4 tables capped at 32 regions (the batched launch for
    d >= 10), a mask is refused exactly when it has more than 32 regions
    (31 ovals or more), and every other code equals the oracle's."""
    edges = I.lift_triangulation(d, 7, noise=1.0)
    exe = _compile(tmp_path, d, G, 32)
    masks = _masks(d, 7, 120)
    got = _run(exe, edges, masks)
    want = oracle.scheme_many(d, edges, masks, threads=4)
    for k in range(len(masks)):
        regions = oracle.n_ovals(oracle.code_int(want[k, 0], want[k, 1])) + 1
        if regions > 32:
            assert got[k, 0] == 0 and got[k, 1] == 1, k   # refused as overflow
        else:
            assert got[k, 0] == want[k, 0] and got[k, 1] == want[k, 1], k
    assert (got[:, 1] == 1).any() and (got[:, 0] != 0).any()
