// jit.cpp -- kernels specialised to one triangulation, built at run time.
//
// For a sweep over billions of sign distributions of one triangulation
// (Sec. 3) the triangulation is a constant.  pw_tri_specialize() writes the
// evaluation of Alg. 1 for that triangulation as straight-line code -- one
// block per diamond vertex with its earlier neighbours and its spanning-tree
// parent as literals, one call per antipodal pair -- compiles it with hipRTC
// for gfx950 and loads it.  The steps it calls (Eval<D>::edge_r, pair,
// vertex3e, finish) and the kernel bodies are the same device functions the
// generic kernels use; only the walk over the program is unrolled, so every
// LDS offset becomes an immediate and no scalar decoding or loop control is
// left.  For sweeps with only sigma(0,0) fixed it also writes the sweep
// evaluator JitSnap: a snapshot of the fixed-sign part shared by the wave
// per chunk of 512 masks (built by label propagation over a per-triangulation
// link table), wave-uniform flags derived from it, a per-chunk reduction of
// what the fixed-sign part leaves to each batch (for even d its antipodal
// pairs, for odd d the crossing tests of its tree edges), and the
// per-batch work on the 9 varying lattice bits.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <sstream>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "patchwork.h"
#include "pw_host.h"
#include "rtc_headers.inc"

namespace pw {

namespace {

// sign of vertex v as an expression: bit p of the mask, flipped by the
// reflection parity g
// (mv: the mask variable; the sweep kernel's per-chunk flags read the
// signs of vertices that are fixed in a chunk from m0, the wave-uniform
// copy of the mask)
std::string sign_expr(const HostProgram& P, int v, const char* mv = "m") {
  const uint32_t rec = P.words[v];
  const int p = rec & 0x7F, g = (rec >> 7) & 1;
  std::string x = std::string("E::bit(") + mv + ", " + std::to_string(p) + ")";
  return g ? "(" + x + " ^ 1u)" : x;
}

// the spanning-tree parent t(v) of the region tree: v's first earlier
// neighbour (-1 for vertex 0)
int tree_parent(const HostProgram& P, int v) { return v > 0 ? (int)P.words[P.nV + (P.words[v] >> 16)] : -1; }

int lattice_bit(const HostProgram& P, int v) { return (int)(P.words[v] & 0x7F); }

constexpr int kAhead = 4;  // phase 3 reads entries this many vertices ahead

// The sweep kernel's tree edges (v, t(v)) with both ends of fixed sign, in
// vertex order (odd d: a chunk reduces their crossing tests).
std::vector<int> fixed_tree_edges(const HostProgram& P, const std::vector<char>& vary) {
  std::vector<int> h;
  for (int v = 0; v < P.nV; ++v) {
    const int t = tree_parent(P, v);
    if (!vary[v] && t >= 0 && !vary[t]) h.push_back(v);
  }
  return h;
}

// phases 2 and 3 and the call of phase 4, common to both evaluators
// pair_stmt(t): the statement of antipodal pair t (empty: the pair is
// already merged in the sweep kernel's snapshot); vary: the sweep kernel's
// varying vertices (null for the plain evaluator).
template <class PairStmt>
void emit_tail(std::ostringstream& o, const HostProgram& P, PairStmt pair_stmt, const std::vector<char>* vary) {
  const int nV = P.nV, nP = P.nP;
  o << "    // phase 2: antipodal pairs\n";
  for (int t = 0; t < nP; ++t) {
    const std::string st = pair_stmt(t);
    if (!st.empty()) o << "    " << st << "\n";
  }
  o << "    // phase 3: region ids and the region tree (each vertex's entry read\n"
       "    // " << kAhead << " vertices ahead)\n";
  o << "    int nR = 0;\n    E::Adj roots = 0;\n";
  // (the sweep kernel reads ahead only the entries of varying vertices: a
  // fixed-sign vertex's entry is read under its flag, which is mostly off)
  for (int v = 0; v < std::min(kAhead, nV); ++v)
    if (!vary || (*vary)[v]) o << "    const uint32_t e" << v << " = E::ent(L, " << v << ");\n";
  if (!vary) {
    for (int v = 0; v < nV; ++v) {
      const int t = tree_parent(P, v);
      if (v + kAhead < nV) o << "    const uint32_t e" << v + kAhead << " = E::ent(L, " << v + kAhead << ");\n";
      o << "    E::vertex3e(L, " << v << ", " << t << ", " << sign_expr(P, v) << ", "
        << (t >= 0 ? sign_expr(P, t) : std::string("0u")) << ", e" << v << ", nR, roots);\n";
    }
    o << "    return E::finish(L, nR, roots, errs);\n";
    return;
  }
  // The sweep kernel.  A vertex of fixed sign whose snapshot entry points
  // to another vertex stays a non-root (the later unions link roots only)
  // and is nobody's parent; its region is that of its snapshot root
  // srow[v].  So region ids are assigned walking only the varying vertices
  // and the snapshot roots (wave-uniform flags fl.fr) in vertex order, a
  // tree parent's region read through its snapshot root; the crossed tree
  // edges of the other vertices (fl.cr: both ends fixed; else per lane) are
  // tested afterwards, with no stores between their loads.
  const bool odd = P.d % 2 == 1;
  auto bitflag = [](const char* w, int v) {
    return std::string("((fl.") + w + "[" + std::to_string(v / 64) + "] >> " + std::to_string(v % 64) + ") & 1u)";
  };
  auto crossed = [&](int v, int t) -> std::string {
    if (!odd || t < 0) return "false";
    if (!(*vary)[v] && !(*vary)[t]) return "(" + bitflag("cr", v) + " != 0u)";
    return "(" + sign_expr(P, v) + " != " + sign_expr(P, t) + ")";
  };
  auto region_of = [&](int x) -> std::string {  // a vertex whose region id is already assigned
    return (*vary)[x] ? std::to_string(x) : "(int)srow[" + std::to_string(x) + "]";
  };
  // Runs of up to 4 consecutive fixed-sign vertices (in one flag word)
  // share one uniform test first: most of them are not snapshot roots.
  // (Entries read ahead for the varying vertices are read before a run.
  // Runs of 4 measured faster than runs of 8 at d = 7.)
  auto run_end = [&](int v0) {
    int v1 = v0;
    while (v1 < nV && !(*vary)[v1] && v1 - v0 < 4 && v1 / 64 == v0 / 64) ++v1;
    return v1;
  };
  auto run_mask = [](int v0, int v1) {
    std::ostringstream h;
    h << "0x" << std::hex << ((1ull << (v1 - v0)) - 1) << "ull";
    return h.str();
  };
  auto read_ahead = [&](int v) {
    if (v + kAhead < nV && (*vary)[v + kAhead])
      o << "    const uint32_t e" << v + kAhead << " = E::ent(L, " << v + kAhead << ");\n";
  };
  auto step3 = [&](int v) {
    const int t = tree_parent(P, v);
    const std::string ev = (*vary)[v] ? "e" + std::to_string(v) : "E::ent(L, " + std::to_string(v) + ")";
    return "E::vertex3c(L, " + std::to_string(v) + ", " + (t >= 0 ? region_of(t) : "-1") + ", " + crossed(v, t) +
           ", " + ev + ", nR, roots);";
  };
  for (int v = 0; v < nV;) {
    if ((*vary)[v]) {
      read_ahead(v);
      o << "    " << step3(v) << "\n";
      ++v;
      continue;
    }
    const int v1 = run_end(v);
    for (int x = v; x < v1; ++x) read_ahead(x);
    if (v1 - v > 1)
      o << "    if ((fl.fr[" << v / 64 << "] >> " << v % 64 << ") & " << run_mask(v, v1) << ") {\n";
    for (int x = v; x < v1; ++x) o << "    if (" << bitflag("fr", x) << ") " << step3(x) << "\n";
    if (v1 - v > 1) o << "    }\n";
    v = v1;
  }
  if (odd) {
    o << "    // crossed tree edges of the fixed-sign non-roots: to a varying\n"
         "    // parent, then between fixed-sign vertices (only the first edge of\n"
         "    // each pair of snapshot roots, runs of 4 edges tested together)\n";
    for (int v = 0; v < nV; ++v) {
      const int t = tree_parent(P, v);
      if ((*vary)[v] || t < 0 || !(*vary)[t]) continue;
      o << "    if (!" << bitflag("fr", v) << ") E::hit(L, srow[" << v << "], " << t << ", " << crossed(v, t)
        << ", roots);\n";
    }
    const std::vector<int> h = fixed_tree_edges(P, *vary);
    const int nh = (int)h.size();
    for (int e = 0; e < nh;) {
      int e1 = e;
      while (e1 < nh && e1 - e < 4 && e1 / 64 == e / 64) ++e1;
      if (e1 - e > 1) o << "    if ((fl.hx[" << e / 64 << "] >> " << e % 64 << ") & " << run_mask(e, e1) << ") {\n";
      for (int x = e; x < e1; ++x)
        o << "    if ((fl.hx[" << x / 64 << "] >> " << x % 64 << ") & 1u) E::hit(L, srow[" << h[x] << "], srow["
          << tree_parent(P, h[x]) << "], true, roots);\n";
      if (e1 - e > 1) o << "    }\n";
      e = e1;
    }
  }
  o << "    return E::finish(L, nR, roots, errs);\n";
}

}  // namespace

// Lattice bits that vary inside one chunk of the sweep kernel with the
// snapshot: the index bits 0 .. 5 + kSnapBits land on mask bits 1 .. 6 +
// kSnapBits when only sigma(0,0) is fixed.
constexpr int kSnapVaryingBits = 6 + 3;

// (d <= 9: the reduction of even d's antipodal pairs needs the varying
// bits to cover the horizontal axis)
bool snapshot_applies(const HostProgram& P) { return P.nA - 1 >= kSnapVaryingBits + 8 && P.d <= kSnapVaryingBits; }

std::string jit_source(const HostProgram& P) {
  std::ostringstream o;
  const int d = P.d, nV = P.nV;
  o << "// generated evaluator for one degree-" << d << " triangulation\n";
  o << "#include \"pw_device.h\"\n\nnamespace pw {\n\nstruct JitEval {\n";
  o << "  __device__ __forceinline__ u128 operator()(Cfg<" << d
    << ">::Mask m, const Lane& L, uint32_t& errs) const {\n";
  o << "    using E = Eval<" << d << ">;\n";
  o << "    E::clear_side(L);\n";
  o << "    // phase 1: components of same-sign vertices; r<u> = a root u had\n";
  for (int v = 0; v < nV; ++v) {
    const uint32_t rec = P.words[v];
    const int n = (rec >> 8) & 0xFF, off = rec >> 16;
    o << "    uint32_t r" << v << " = " << v << "u; { const uint32_t sv = " << sign_expr(P, v) << ";";
    for (int k = 0; k < n; ++k) {
      const int u = (int)P.words[nV + off + k];
      o << " E::edge_r(L, sv, " << sign_expr(P, u) << ", " << v << ", r" << v << ", r" << u << ");";
    }
    o << " E::close(L, " << v << ", r" << v << "); }\n";
  }
  emit_tail(
      o, P,
      [&](int t) {
        const uint32_t pr = P.words[nV + P.nE + t];
        return "E::pair(L, " + std::to_string(pr & 0xFFFF) + ", " + std::to_string(pr >> 16) + ");";
      },
      nullptr);
  o << "  }\n};\n\n";
  if (snapshot_applies(P)) {
    // vertices whose sign varies inside a chunk, and the full adjacency
    std::vector<char> vary(nV, 0);
    std::vector<std::vector<int>> adj(nV);
    for (int v = 0; v < nV; ++v) {
      const int b = lattice_bit(P, v);
      vary[v] = (b >= 1 && b <= kSnapVaryingBits) ? 1 : 0;
      const uint32_t rec = P.words[v];
      const int n = (rec >> 8) & 0xFF, off = rec >> 16;
      for (int k = 0; k < n; ++k) {
        const int u = (int)P.words[nV + off + k];
        adj[v].push_back(u);
        adj[u].push_back(v);
      }
    }
    // The snapshot: the components of the fixed-sign part (for odd d with
    // the antipodal pairs of fixed-sign vertices merged too: that is a plain
    // union, and the regions do not depend on the order of unions).  Every
    // lane would compute the same union-find, so the wave shares one label
    // row instead: lane l owns the vertices l + 64 k, and min-label
    // propagation with pointer jumping over the links below reaches, for
    // each vertex, the smallest vertex of its component -- the root the
    // union-find would give (links always point to the smaller root).  A
    // varying vertex (and the padding after vertex NV-1) keeps its own
    // index, its entry before its edges are added.
    const int nE = P.nE;
    const bool even = d % 2 == 0;
    auto both_fixed = [&](int t) {
      const uint32_t pr = P.words[nV + nE + t];
      return !vary[pr & 0xFFFF] && !vary[pr >> 16];
    };
    auto fixed_pair = [&](int t) { return !even && both_fixed(t); };
    const int nw = (nV + 63) / 64;
    // links of each fixed-sign vertex: same-sign neighbours (packed: u,
    // lattice bits of u and v, flip difference) and antipodal partners
    std::vector<std::vector<uint32_t>> links(nV);
    auto bit_of = [&](int x) { return (uint32_t)lattice_bit(P, x); };
    auto flip_of = [&](int x) { return (uint32_t)((P.words[x] >> 7) & 1); };
    for (int v = 0; v < nV; ++v) {
      if (vary[v]) continue;
      for (int u : adj[v])
        if (!vary[u])
          links[v].push_back((uint32_t)u | bit_of(u) << 8 | (flip_of(u) ^ flip_of(v)) << 15 | bit_of(v) << 16 | 1u << 24);
    }
    for (int t = 0; t < P.nP; ++t)
      if (fixed_pair(t)) {
        const uint32_t pr = P.words[nV + nE + t];
        const int a = (int)(pr & 0xFFFF), b = (int)(pr >> 16);
        links[a].push_back((uint32_t)b | 1u << 23 | 1u << 24);
        links[b].push_back((uint32_t)a | 1u << 23 | 1u << 24);
      }
    size_t slots = 1;
    for (const auto& l : links) slots = std::max(slots, l.size());
    o << "// per owned vertex (lane + 64 k) and slot: bits 0-7 the linked vertex,\n"
         "// 8-14 its lattice bit, 15 the flip difference, 16-22 the owner's\n"
         "// lattice bit, 23 unconditional (antipodal pair), 24 present\n";
    o << "__device__ const uint32_t kSnapLinks[" << nw * 64 * slots << "] = {";
    for (int v = 0; v < nw * 64; ++v)
      for (size_t j = 0; j < slots; ++j) {
        const uint32_t x = (v < nV && j < links[v].size()) ? links[v][j] : 0u;
        o << (v || j ? "," : "") << (j == 0 ? "\n  " : " ") << "0x" << std::hex << x << std::dec << "u";
      }
    o << "};\n";
    if (d % 2 == 1) {
      const std::vector<int> he = fixed_tree_edges(P, vary);
      o << "// per tree edge between fixed-sign vertices: bits 0-7 v, 8-15 t(v), 16-22\n"
           "// v's lattice bit, 23-29 t's, 30 the flip difference\n";
      o << "__device__ const uint32_t kHitEdges[" << std::max<size_t>(1, he.size()) << "] = {";
      for (size_t e = 0; e < std::max<size_t>(1, he.size()); ++e) {
        uint32_t x = 0;
        if (e < he.size()) {
          const int v = he[e], t = tree_parent(P, v);
          x = (uint32_t)v | (uint32_t)t << 8 | bit_of(v) << 16 | bit_of(t) << 23 | (flip_of(v) ^ flip_of(t)) << 30;
        }
        o << (e ? "," : "") << (e % 8 == 0 ? "\n  " : " ") << "0x" << std::hex << x << std::dec << "u";
      }
      o << "};\n";
    }
    o << "struct JitSnap {\n  using E = Eval<" << d << ">;\n";
    o << "  static constexpr int kNW = " << nw << ", kSlots = " << slots << ";\n";
    o << "  static constexpr int kRow = Cfg<" << d << ">::SNAP_WORDS * 4 / Cfg<" << d << ">::EB;\n";
    o << "  // the row offsets a lane takes the minimum over (its own vertex where\n"
         "  // a link is absent or inactive in this chunk)\n";
    o << "  struct Links {\n    uint32_t a[kNW][kSlots];\n  };\n";
    o << "  __device__ __forceinline__ static void snap_init(uint8_t* snap, int lane) {\n"
         "    E::Ent* row = reinterpret_cast<E::Ent*>(snap);\n"
         "    for (int k = 0; k < kNW; ++k) {\n      const int v = lane + 64 * k;\n"
         "      if (v < kRow) row[v] = (E::Ent)v;\n    }\n  }\n";
    o << "  __device__ __forceinline__ static Links snap_links(uint64_t m0, int lane) {\n    Links ln;\n"
         "    for (int k = 0; k < kNW; ++k) {\n      const uint32_t v = (uint32_t)(lane + 64 * k);\n"
         "      for (int j = 0; j < kSlots; ++j) {\n"
         "        const uint32_t x = kSnapLinks[v * kSlots + j];\n"
         "        const uint32_t same = (uint32_t)((m0 >> ((x >> 8) & 0x7F)) ^ (m0 >> ((x >> 16) & 0x7F))) & 1u;\n"
         "        const bool on = ((x >> 24) & 1u) && (((x >> 23) & 1u) || same == ((x >> 15) & 1u));\n"
         "        ln.a[k][j] = on ? (x & 0xFFu) : v;\n      }\n    }\n    return ln;\n  }\n";
    o << "  // one round over the lane's vertices; true if a label went down\n";
    o << "  __device__ __forceinline__ static bool snap_step(const Links& ln, uint8_t* snap, int lane) {\n"
         "    E::Ent* row = reinterpret_cast<E::Ent*>(snap);\n    bool changed = false;\n"
         "    for (int k = 0; k < kNW; ++k) {\n      const int v = lane + 64 * k;\n"
         "      if (v >= Cfg<" << d << ">::NV) continue;\n"
         "      const uint32_t cur = row[v];\n      uint32_t mn = cur;\n"
         "      for (int j = 0; j < kSlots; ++j) {\n        const uint32_t y = row[ln.a[k][j]];\n"
         "        mn = y < mn ? y : mn;\n      }\n"
         "      const uint32_t z = row[mn];  // pointer jumping: a label's own label is no larger\n"
         "      mn = z < mn ? z : mn;\n"
         "      if (mn < cur) {\n        row[v] = (E::Ent)mn;\n        changed = true;\n      }\n    }\n"
         "    return changed;\n  }\n";
    if (even) {
      // Even d: the antipodal pairs of fixed-sign vertices carry a parity
      // (they join opposite sides), which the plain label propagation
      // cannot merge.  They are reduced per chunk instead.  Stage 1: each
      // lane applies them, in order, to its own copy of the snapshot row; a
      // pair that joins two sets belongs to a spanning forest of the pairs
      // over the snapshot's sets, one that first closes an odd cycle of a
      // set marks it, and any other changes nothing in any batch (the
      // cycle it closes has the parity of the forest path, or the set is
      // marked already).  Stages 2 and 3: the sets of the pair graph that
      // no varying vertex reaches -- none of their vertices has a varying
      // neighbour or partner, so no phase-1 edge or pair of a batch touches
      // them -- are merged into the snapshot row, each vertex pointing at
      // the set's smallest vertex (the root the union-find would give).
      // Such a set has no odd cycle: the varying bits 1 .. 9 include the
      // lattice points (i, 0), i = 1 .. d (bits 1 .. d in the bit order;
      // the sweep kernel exists for d <= 9), so the varying vertices cover
      // the horizontal axis line of the reflected diamond but its centre,
      // a one-sided loop that every other one crosses; a cycle of
      // fixed-sign vertices closed by an odd number of pairs is one-sided,
      // so it passes through the centre, whose neighbours (1, 0) and
      // (0, 1) vary.  Only the forest pairs and marks of the reached sets
      // are left to each batch.
      std::vector<uint64_t> touch(nw, 0), fixedv(nw, 0);
      for (int v = 0; v < nV; ++v) {
        if (vary[v]) continue;
        fixedv[v / 64] |= 1ull << (v % 64);
        for (int u : adj[v])
          if (vary[u]) touch[v / 64] |= 1ull << (v % 64);
      }
      for (int t = 0; t < P.nP; ++t) {
        const uint32_t pr = P.words[nV + nE + t];
        const int a = (int)(pr & 0xFFFF), b = (int)(pr >> 16);
        if (vary[a] && !vary[b]) touch[b / 64] |= 1ull << (b % 64);
        if (vary[b] && !vary[a]) touch[a / 64] |= 1ull << (a % 64);
      }
      // (bit lane of word k: vertex lane + 64 k, the one the lane owns)
      auto lit = [](uint64_t x) {
        std::ostringstream h;
        h << "0x" << std::hex << x << "ull";
        return h.str();
      };
      const std::string C = "Cfg<" + std::to_string(d) + ">::";
      o << "  __device__ __forceinline__ static uint64_t pairs_1(const Lane& L, uint8_t* snap, int lane) {\n"
           "    uint32_t* w = reinterpret_cast<uint32_t*>(snap);\n"
           "    for (int k = 0; k < " << C << "SNAP_WORDS; ++k) L.eword(k) = w[k];\n"
           "    E::clear_side(L);\n    uint32_t kf = 0, ko = 0;\n";
      for (int t = 0; t < P.nP; ++t) {
        if (!both_fixed(t)) continue;
        const uint32_t pr = P.words[nV + nE + t];
        o << "    { const uint32_t k = E::pair_kind(L, " << (pr & 0xFFFF) << ", " << (pr >> 16)
          << "); kf |= (uint32_t)(k == 1u) << " << t << "; ko |= (uint32_t)(k == 2u) << " << t << "; }\n";
      }
      o << "    if (lane < " << C << "TOUCH_WORDS) w[" << C << "SNAP_TOUCH + lane] = 0;\n"
           "    return (uint64_t)kf | (uint64_t)ko << 32;\n  }\n";
      o << "  __device__ __forceinline__ static void pairs_2(const Lane& L, uint8_t* snap, int lane) {\n"
           "    // the sets that vertices with a varying neighbour or partner are in\n"
           "    uint32_t* w = reinterpret_cast<uint32_t*>(snap);\n";
      for (int k = 0; k < nw; ++k)
        o << "    if ((" << lit(touch[k]) << " >> lane) & 1u) {\n"
             "      const uint32_t r = E::root_of(L, (uint32_t)(lane + " << 64 * k << "));\n"
             "      atomicOr(&w[" << C << "SNAP_TOUCH + (r >> 5)], 1u << (r & 31u));\n    }\n";
      o << "  }\n";
      o << "  __device__ __forceinline__ static void pairs_3(const Lane& L, uint8_t* snap, int lane, uint64_t kinds) {\n"
           "    uint32_t* w = reinterpret_cast<uint32_t*>(snap);\n"
           "    E::Ent* row = reinterpret_cast<E::Ent*>(snap);\n"
           "    auto reached = [&](uint32_t r) { return (w[" << C << "SNAP_TOUCH + (r >> 5)] >> (r & 31u)) & 1u; };\n"
           "    // the lane's fixed-sign vertices in sets no varying vertex reaches\n";
      for (int k = 0; k < nw; ++k)
        o << "    if ((" << lit(fixedv[k]) << " >> lane) & 1u) {\n"
             "      const uint32_t v = (uint32_t)(lane + " << 64 * k << "), r = E::root_of(L, v);\n"
             "      if (!reached(r) && row[v] != r) row[v] = (E::Ent)r;\n    }\n";
      o << "    // the pairs of the other sets\n    uint32_t keep = 0;\n";
      for (int t = 0; t < P.nP; ++t) {
        if (!both_fixed(t)) continue;
        const uint32_t pr = P.words[nV + nE + t];
        o << "    keep |= reached(E::root_of(L, " << (pr & 0xFFFF) << "u)) << " << t << ";\n";
      }
      o << "    w[" << C << "SNAP_KIND] = (uint32_t)kinds & keep;\n"
           "    w[" << C << "SNAP_KIND + 1] = (uint32_t)(kinds >> 32) & keep;\n  }\n";
    }
    const std::vector<int> hedges = fixed_tree_edges(P, vary);
    const int nh = (int)hedges.size(), nhk = (nh + 63) / 64, nh32 = (nh + 31) / 32;
    if (!even) {
      // Odd d: a crossed tree edge between two fixed-sign non-root and
      // parent vertices marks the root region when its two snapshot roots
      // end up in one region; every edge with the same pair of snapshot
      // roots tests the same thing (about 34 such edges per batch over 6
      // pairs at d = 7).  Per chunk, stage 1 writes each edge's pair (a key;
      // none if the edge is not crossed or v is a snapshot root) and stage 2
      // keeps the first edge of each key; a batch tests only those.
      o << "  static constexpr int kNH = " << nh << ", kHK = " << nhk << ";\n";
      o << "  __device__ __forceinline__ static void hits_1(uint8_t* snap, int lane, uint64_t m0) {\n"
           "    uint32_t* w = reinterpret_cast<uint32_t*>(snap);\n"
           "    const E::Ent* row = reinterpret_cast<const E::Ent*>(snap);\n"
           "    uint16_t* key = reinterpret_cast<uint16_t*>(w + Cfg<" << d << ">::SNAP_HKEY);\n"
           "    if (lane < Cfg<" << d << ">::HIT_WORDS) w[Cfg<" << d << ">::SNAP_HX + lane] = 0;\n"
           "    for (int k = 0; k < kHK; ++k) {\n"
           "      const int e = lane + 64 * k;\n"
           "      if (e >= kNH) continue;\n"
           "      const uint32_t x = kHitEdges[e], v = x & 0xFFu, t = (x >> 8) & 0xFFu;\n"
           "      const uint32_t a = row[v], b = row[t];\n"
           "      const bool crossed = ((uint32_t)((m0 >> ((x >> 16) & 0x7Fu)) ^ (m0 >> ((x >> 23) & 0x7Fu))) ^ (x >> 30)) & 1u;\n"
           "      const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;\n"
           "      key[e] = (uint16_t)((a != v && crossed) ? (lo | hi << 8) : 0xFFFFu);\n"
           "    }\n  }\n";
      o << "  __device__ __forceinline__ static void hits_2(uint8_t* snap, int lane) {\n"
           "    uint32_t* w = reinterpret_cast<uint32_t*>(snap);\n"
           "    const uint16_t* key = reinterpret_cast<const uint16_t*>(w + Cfg<" << d << ">::SNAP_HKEY);\n"
           "    for (int k = 0; k < kHK; ++k) {\n"
           "      const int e = lane + 64 * k;\n"
           "      const uint32_t my = e < kNH ? (uint32_t)key[e] : 0xFFFFu;\n"
           "      bool first = my != 0xFFFFu;\n"
           "      const int jn = kNH < 64 * (k + 1) ? kNH : 64 * (k + 1);\n"
           "      for (int j = 0; j < jn; ++j) first = first && !(j < e && (uint32_t)key[j] == my);\n"
           "      if (first) atomicOr(&w[Cfg<" << d << ">::SNAP_HX + (e >> 5)], 1u << (e & 31));\n"
           "    }\n  }\n";
    }
    o << "  __device__ __forceinline__ void snapshot(Cfg<" << d
      << ">::Mask m, const Lane& L, uint8_t* snap, int lane) const {\n"
         "    (void)L;\n    snap_init(snap, lane);\n    const Links ln = snap_links(uniform_mask(m), lane);\n"
         "    // labels only go down: at most NV rounds (the bound is never reached)\n"
         "    for (int round = 0; round <= Cfg<"
      << d << ">::NV; ++round)\n      if (__builtin_amdgcn_ballot_w64(snap_step(ln, snap, lane)) == 0) break;\n";
    if (even)
      o << "    // the stages read what other lanes wrote in the one before\n"
           "    PW_FENCE();\n    __builtin_amdgcn_wave_barrier();\n    const uint64_t kinds = pairs_1(L, snap, lane);\n"
           "    PW_FENCE();\n    __builtin_amdgcn_wave_barrier();\n    pairs_2(L, snap, lane);\n"
           "    PW_FENCE();\n    __builtin_amdgcn_wave_barrier();\n    pairs_3(L, snap, lane, kinds);\n"
           "    PW_FENCE();\n";
    else
      o << "    // the stages read what other lanes wrote in the one before\n"
           "    PW_FENCE();\n    __builtin_amdgcn_wave_barrier();\n    hits_1(snap, lane, uniform_mask(m));\n"
           "    PW_FENCE();\n    __builtin_amdgcn_wave_barrier();\n    hits_2(snap, lane);\n"
           "    PW_FENCE();\n";
    o << "  }\n";
    // The edges of phase 1 between a varying vertex and a fixed-sign
    // neighbour, in the order the batch adds them; such an edge is a
    // duplicate when an earlier fixed-sign neighbour of the same vertex has
    // the same snapshot root and the same sign (for odd d the antipodal
    // pairs merged in the snapshot may join vertices of both signs): its
    // union changes nothing.
    std::vector<std::vector<int>> earlier_fixed;  // per edge: the earlier fixed neighbours
    std::vector<int> edge_u;
    for (int v = 0; v < nV; ++v) {
      if (!vary[v]) continue;
      std::vector<int> nb = adj[v];
      std::sort(nb.begin(), nb.end());
      std::vector<int> seen;
      for (int u : nb) {
        if (vary[u]) continue;
        earlier_fixed.push_back(seen);
        edge_u.push_back(u);
        seen.push_back(u);
      }
    }
    const int n_fixed_edges = (int)edge_u.size();
    const int nd = std::max(1, (n_fixed_edges + 63) / 64);
    // the wave-uniform flags of a chunk, from the snapshot row (entry v
    // is v: v is a root of the fixed-sign part) and from m0
    o << "  struct Flags {\n    uint64_t fr[" << nw << "];  // fixed-sign vertices that are snapshot roots\n"
      << "    uint64_t cr[" << nw << "];  // fixed-sign vertices whose tree edge (both ends fixed) is crossed\n"
      << "    uint64_t dp[" << nd << "];  // duplicate phase-1 edges to fixed-sign neighbours\n";
    if (even) o << "    uint32_t fp, op;  // fixed-sign pairs left to each batch: joining two sets, marking one\n";
    else o << "    uint64_t hx[" << std::max(1, nhk) << "];  // fixed-sign tree edges whose crossing a batch tests\n";
    o << "  };\n";
    o << "  __device__ __forceinline__ Flags flags(Cfg<" << d << ">::Mask m0, const uint8_t* snap) const {\n";
    o << "    Flags fl{};\n    const E::Ent* row = reinterpret_cast<const E::Ent*>(snap);\n";
    for (int v = 0; v < nV; ++v)
      if (!vary[v]) o << "    const uint32_t w" << v << " = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)row[" << v << "]);\n";
    for (int e = 0; e < n_fixed_edges; ++e) {
      if (earlier_fixed[e].empty()) continue;
      o << "    fl.dp[" << e / 64 << "] |= (uint64_t)(";
      for (size_t k = 0; k < earlier_fixed[e].size(); ++k)
        o << (k ? " || " : "") << "(w" << edge_u[e] << " == w" << earlier_fixed[e][k] << " && "
          << sign_expr(P, edge_u[e], "m0") << " == " << sign_expr(P, earlier_fixed[e][k], "m0") << ")";
      o << ") << " << e % 64 << ";\n";
    }
    for (int v = 0; v < nV; ++v) {
      if (vary[v]) continue;
      o << "    fl.fr[" << v / 64 << "] |= (uint64_t)(w" << v << " == " << v << "u) << " << v % 64 << ";\n";
      const int t = tree_parent(P, v);
      if (d % 2 == 1 && t >= 0 && !vary[t])
        o << "    fl.cr[" << v / 64 << "] |= (uint64_t)(" << sign_expr(P, v, "m0") << " ^ " << sign_expr(P, t, "m0")
          << ") << " << v % 64 << ";\n";
    }
    if (!even)
      for (int k = 0; k < nh32; ++k)
        o << "    fl.hx[" << k / 2 << "] |= (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(reinterpret_cast<const "
             "uint32_t*>(snap)[Cfg<" << d << ">::SNAP_HX + " << k << "]) << " << 32 * (k % 2) << ";\n";
    if (even)
      o << "    fl.fp = (uint32_t)__builtin_amdgcn_readfirstlane(reinterpret_cast<const uint32_t*>(snap)[Cfg<" << d
        << ">::SNAP_KIND]);\n    fl.op = (uint32_t)__builtin_amdgcn_readfirstlane(reinterpret_cast<const uint32_t*>(snap)[Cfg<"
        << d << ">::SNAP_KIND + 1]);\n";
    o << "    return fl;\n  }\n";
    o << "  // one batch: restore, the edges of the varying vertices, then as usual\n";
    o << "  __device__ __forceinline__ u128 batch(Cfg<" << d
      << ">::Mask m, const Lane& L, const uint8_t* snap, const Flags& fl_chunk, uint32_t& errs) const {\n";
    // (the flags pass through an opaque copy per batch: tests of single
    // flag bits hoisted out of the batch loop would each hold a register)
    o << "    Flags fl;\n";
    for (int k = 0; k < nw; ++k)
      o << "    { uint64_t a = fl_chunk.fr[" << k << "], b = fl_chunk.cr[" << k
        << "]; PW_OPAQUE(a); PW_OPAQUE(b); fl.fr[" << k << "] = uniform_mask(a); fl.cr[" << k
        << "] = uniform_mask(b); }\n";
    for (int k = 0; k < nd; ++k)
      o << "    { uint64_t a = fl_chunk.dp[" << k << "]; PW_OPAQUE(a); fl.dp[" << k << "] = uniform_mask(a); }\n";
    if (!even)
      for (int k = 0; k < std::max(1, nhk); ++k)
        o << "    { uint64_t a = fl_chunk.hx[" << k << "]; PW_OPAQUE(a); fl.hx[" << k << "] = uniform_mask(a); }\n";
    if (even)
      o << "    { uint32_t a = fl_chunk.fp, b = fl_chunk.op; PW_OPAQUE(a); PW_OPAQUE(b); "
           "fl.fp = (uint32_t)__builtin_amdgcn_readfirstlane(a); fl.op = (uint32_t)__builtin_amdgcn_readfirstlane(b); }\n";
    // the restore: the row, a word at a time (a compiler barrier every 8
    // words keeps the loads from all being hoisted at once, which would
    // need a register each)
    o << "    {\n      const uint32_t* s = reinterpret_cast<const uint32_t*>(__builtin_assume_aligned(snap, 16));\n"
         "#pragma unroll\n      for (int k = 0; k < Cfg<"
      << d << ">::SNAP_WORDS; ++k) {\n        L.eword(k) = s[k];\n        if (k % 8 == 7) PW_FENCE();\n      }\n";
    o << "    }\n    E::clear_side(L);\n";
    o << "    const E::Ent* srow = reinterpret_cast<const E::Ent*>(snap);\n";
    o << "    // phase 1 for the varying vertices (in index order; each with all\n"
         "    // its fixed-sign neighbours and its earlier varying ones; duplicate\n"
         "    // edges skipped)\n";
    int fe = 0;  // the next edge to a fixed-sign neighbour
    for (int v = 0; v < nV; ++v) {
      if (!vary[v]) continue;
      o << "    uint32_t r" << v << " = " << v << "u; { const uint32_t sv = " << sign_expr(P, v) << ";";
      std::vector<int> nb = adj[v];
      std::sort(nb.begin(), nb.end());
      // the fixed-sign neighbours' snapshot roots (wave-uniform), all read
      // before the first union so that their loads overlap
      for (int u : nb)
        if (!vary[u]) o << " const uint32_t s" << u << " = srow[" << u << "];";
      for (int u : nb) {
        if (vary[u] && u > v) continue;
        if (vary[u]) {
          o << " E::edge_v(L, sv, " << sign_expr(P, u) << ", " << v << ", r" << v << ", r" << u << ");";
        } else {
          const std::string step = "{ uint32_t t = s" + std::to_string(u) + "; E::edge_v(L, sv, " +
                                   sign_expr(P, u) + ", " + std::to_string(v) + ", r" + std::to_string(v) + ", t); }";
          if (earlier_fixed[fe].empty())
            o << " " << step;
          else
            o << " if (!((fl.dp[" << fe / 64 << "] >> " << fe % 64 << ") & 1u)) " << step;
          ++fe;
        }
      }
      o << " }\n";
    }
    emit_tail(
        o, P,
        [&](int t) -> std::string {
          const uint32_t pr = P.words[nV + nE + t];
          const std::string a = std::to_string(pr & 0xFFFF), b = std::to_string(pr >> 16), ts = std::to_string(t);
          if (fixed_pair(t)) return "";
          if (even && both_fixed(t))
            return "if ((fl.fp >> " + ts + ") & 1u) E::pair(L, (int)srow[" + a + "], (int)srow[" + b +
                   "]); else if ((fl.op >> " + ts + ") & 1u) E::odd_mark(L, (int)srow[" + a + "]);";
          return "E::pair(L, " + a + ", " + b + ");";
        },
        &vary);
    o << "  }\n};\n\n";
  }
  o << "}  // namespace pw\n\n";
  const std::string attr = "extern \"C\" __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(pw::Cfg<" +
                           std::to_string(d) + ">::WAVES_PER_EU))) void ";
  o << attr << "pw_jit_codes(const void* masks, int64_t n, uint64_t* codes, uint32_t* errflag) {\n"
       "  extern __shared__ uint32_t smem[];\n  pw::codes_body<"
    << d << ">(pw::JitEval{}, masks, n, codes, errflag, smem);\n}\n";
  o << attr << "pw_jit_hist(const void* masks, int64_t n, uint64_t index_base, const pw::HistDev* h, "
       "uint64_t* codes, uint32_t* errflag) {\n  extern __shared__ uint32_t smem[];\n  pw::hist_body<"
    << d << ">(pw::JitEval{}, masks, n, index_base, h, codes, errflag, smem);\n}\n";
  o << attr << "pw_jit_enum(uint64_t first, uint64_t count, pw::Runs runs, const pw::HistDev* h, "
       "uint32_t* errflag) {\n  extern __shared__ uint32_t smem[];\n  pw::enum_body<"
    << d << ">(pw::JitEval{}, first, count, runs, h, errflag, smem);\n}\n";
  if (snapshot_applies(P))
    o << attr << "pw_jit_enum_snap(uint64_t first, uint64_t count, pw::Runs runs, const pw::HistDev* h, "
         "uint32_t* errflag) {\n  extern __shared__ uint32_t smem[];\n  pw::enum_snap_body<"
      << d << ">(pw::JitSnap{}, first, count, runs, h, errflag, smem);\n}\n";
  return o.str();
}

namespace {

const char* const kRtcNames[] = {kRtcHeaderName0, kRtcHeaderName1};
const char* const kRtcTexts[] = {kRtcHeaderText0, kRtcHeaderText1};

// hipRTC options: gfx950, no packed FP32 instructions (as for the library)
const char* const kRtcOptions[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                                   "-Xclang", "-packed-fp32-ops"};

pw_status compile(const std::string& src, std::vector<char>* code) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "pw_jit.hip", kRtcHeaderCount, kRtcTexts, kRtcNames) !=
      HIPRTC_SUCCESS)
    return set_err(PW_ERR_HIP, "hiprtcCreateProgram failed");
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof kRtcOptions / sizeof *kRtcOptions), kRtcOptions);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n + 1, '\0');
    hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    return set_err(PW_ERR_HIP, "hipRTC compile failed: %.400s", log.c_str());
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  code->resize(n);
  hiprtcGetCode(prog, code->data());
  hiprtcDestroyProgram(&prog);
  return PW_OK;
}

}  // namespace
}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_jit_source(int32_t d, const int16_t* edges_ij, int32_t n_edges, char* buf, int64_t cap, int64_t* len) {
  if (!len) return set_err(PW_ERR_ARG, "null argument");
  static thread_local HostProgram P;
  char msg[256];
  const int rc = build_program(d, edges_ij, n_edges, &P, msg, sizeof msg);
  if (rc != 0) return set_err(rc, "%s", msg);
  const std::string s = jit_source(P);
  *len = (int64_t)s.size();
  if (buf && cap > 0) {
    const int64_t n = std::min<int64_t>(cap - 1, (int64_t)s.size());
    std::memcpy(buf, s.data(), (size_t)n);
    buf[n] = '\0';
  }
  return PW_OK;
}

pw_status pw_jit_compile(int32_t d, const int16_t* edges_ij, int32_t n_edges, int64_t* code_bytes) {
  if (d > kJitMaxDegree) return set_err(PW_ERR_ARG, "specialised kernels exist for d <= %d", kJitMaxDegree);
  static thread_local HostProgram P;
  char msg[256];
  const int brc = build_program(d, edges_ij, n_edges, &P, msg, sizeof msg);
  if (brc != 0) return set_err(brc, "%s", msg);
  std::vector<char> code;
  const pw_status rc = compile(jit_source(P), &code);
  if (rc == PW_OK && code_bytes) *code_bytes = (int64_t)code.size();
  return rc;
}

pw_status pw_tri_specialize(pw_tri_t t) {
  if (!t) return set_err(PW_ERR_ARG, "null handle");
  if (t->prog.d > kJitMaxDegree) return set_err(PW_ERR_ARG, "specialised kernels exist for d <= %d", kJitMaxDegree);
  if (t->jit_mod) return PW_OK;
  // Code objects are kept per source text for the life of the process: a
  // triangulation equal to an earlier one (same edges, hence the same
  // generated source) loads the kept object instead of compiling again.
  // Each handle still loads its own module and runs its own launches.
  static std::mutex cache_mu;
  static std::map<std::string, std::vector<char>> cache;
  const std::string src = jit_source(t->prog);
  std::vector<char> code;
  {
    std::lock_guard<std::mutex> lock(cache_mu);
    const auto it = cache.find(src);
    if (it != cache.end()) code = it->second;
  }
  if (code.empty()) {
    const pw_status rc = compile(src, &code);
    if (rc != PW_OK) return rc;
    std::lock_guard<std::mutex> lock(cache_mu);
    if (cache.size() >= 256) cache.clear();  // bound the host memory it holds
    cache.emplace(src, code);
  }
  hipModule_t mod = nullptr;
  PW_HIP(hipModuleLoadData(&mod, code.data()));
  hipFunction_t fc = nullptr, fh = nullptr, fe = nullptr, fs = nullptr;
  hipError_t e = hipModuleGetFunction(&fc, mod, "pw_jit_codes");
  if (e == hipSuccess) e = hipModuleGetFunction(&fh, mod, "pw_jit_hist");
  if (e == hipSuccess) e = hipModuleGetFunction(&fe, mod, "pw_jit_enum");
  if (e == hipSuccess && snapshot_applies(t->prog)) e = hipModuleGetFunction(&fs, mod, "pw_jit_enum_snap");
  if (e != hipSuccess) {
    (void)hipModuleUnload(mod);
    return set_err(PW_ERR_HIP, "%s (code %d)", hipGetErrorString(e), (int)e);
  }
  t->jit_mod = mod;
  t->jit_codes = fc;
  t->jit_hist = fh;
  t->jit_enum = fe;
  t->jit_enum_snap = fs;
  return PW_OK;
}

}  // extern "C"
