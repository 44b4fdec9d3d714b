// tri.cpp -- host side of pw_tri_create: validate an edge list as a
// unimodular triangulation of d*Delta_2 (Sec. 2) and build the reflected
// diamond program that the kernels walk (Alg. 1, first two steps).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <utility>
#include <vector>

#include "pw_internal.h"

namespace pw {
namespace {

using Pt = std::pair<int, int>;

int fail(char* err, int errlen, int code, const char* msg) {
  std::snprintf(err, errlen, "%s", msg);
  return code;
}

int point_index(int d, int i, int j) { return j * (d + 1) - j * (j - 1) / 2 + i; }

bool in_lattice(int d, int i, int j) { return i >= 0 && j >= 0 && i + j <= d; }

int gcd_abs(int a, int b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  while (b) {
    int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

long cross(Pt a, Pt b, Pt c) {
  return (long)(b.first - a.first) * (c.second - a.second) - (long)(b.second - a.second) * (c.first - a.first);
}

// both ends on one side of the big triangle
bool on_boundary(int d, Pt a, Pt b) {
  return (a.second == 0 && b.second == 0) || (a.first == 0 && b.first == 0) ||
         (a.first + a.second == d && b.first + b.second == d);
}

}  // namespace

int build_program(int d, const int16_t* edges_ij, int n_edges, HostProgram* prog, char* err, int errlen) {
  const int kArg = -1, kTri = -2;
  if (d < 1 || d > kDMax) return fail(err, errlen, kArg, "degree must be in [1, 12]");
  if (!edges_ij || !prog) return fail(err, errlen, kArg, "null pointer");
  const int nA = n_points(d);
  if (n_edges != nA + d * d - 1) {
    char m[160];
    std::snprintf(m, sizeof m, "a unimodular triangulation of %d*Delta_2 has %d edges, got %d", d,
                  nA + d * d - 1, n_edges);
    return fail(err, errlen, kTri, m);
  }
  // --- the edge list ---
  std::set<std::pair<Pt, Pt>> edge_set;
  std::map<Pt, std::set<Pt>> nbr;
  std::vector<std::pair<Pt, Pt>> edges;
  for (int k = 0; k < n_edges; ++k) {
    Pt a{edges_ij[4 * k], edges_ij[4 * k + 1]}, b{edges_ij[4 * k + 2], edges_ij[4 * k + 3]};
    if (!in_lattice(d, a.first, a.second) || !in_lattice(d, b.first, b.second))
      return fail(err, errlen, kTri, "edge endpoint outside A");
    if (gcd_abs(b.first - a.first, b.second - a.second) != 1)
      return fail(err, errlen, kTri, "edge is not primitive");
    if (b < a) std::swap(a, b);
    if (!edge_set.insert({a, b}).second) return fail(err, errlen, kTri, "repeated edge");
    nbr[a].insert(b);
    nbr[b].insert(a);
    edges.push_back({a, b});
  }
  // --- triangles: unimodular 3-cliques ---
  std::map<std::pair<Pt, Pt>, std::vector<Pt>> apex;  // edge -> third vertices
  int n_tri = 0;
  for (auto& e : edges) {
    for (const Pt& c : nbr[e.first]) {
      if (!(e.second < c) || !nbr[e.second].count(c)) continue;
      long D = cross(e.first, e.second, c);
      if (D != 1 && D != -1) continue;
      ++n_tri;
      Pt tri[3] = {e.first, e.second, c};
      for (int s = 0; s < 3; ++s) {
        Pt u = tri[s], v = tri[(s + 1) % 3], w = tri[(s + 2) % 3];
        if (v < u) std::swap(u, v);
        apex[{u, v}].push_back(w);
      }
    }
  }
  if (n_tri != d * d) return fail(err, errlen, kTri, "the edges do not form d^2 unimodular triangles");
  for (auto& e : edges) {
    auto it = apex.find(e);
    int cnt = it == apex.end() ? 0 : (int)it->second.size();
    if (on_boundary(d, e.first, e.second)) {
      if (cnt != 1) return fail(err, errlen, kTri, "a boundary edge must lie in exactly one triangle");
    } else {
      if (cnt != 2) return fail(err, errlen, kTri, "an interior edge must lie in exactly two triangles");
      long s0 = cross(e.first, e.second, it->second[0]), s1 = cross(e.first, e.second, it->second[1]);
      if ((s0 > 0) == (s1 > 0)) return fail(err, errlen, kTri, "the two triangles of an edge overlap");
    }
  }
  // --- the diamond A<>: rows y = -d..d, x ascending ---
  const int side = 2 * d + 1;
  std::vector<int> id(side * side, -1);
  std::vector<Pt> vert;
  for (int y = -d; y <= d; ++y)
    for (int x = -d; x <= d; ++x)
      if (std::abs(x) + std::abs(y) <= d) {
        id[(y + d) * side + (x + d)] = (int)vert.size();
        vert.push_back({x, y});
      }
  auto vid = [&](int x, int y) { return id[(y + d) * side + (x + d)]; };
  const int nV = (int)vert.size();
  // E(T<>): the four reflections of every edge, as a set
  std::set<std::pair<int, int>> dedges;
  const int eps[4][2] = {{1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
  for (auto& e : edges)
    for (auto& q : eps) {
      int a = vid(q[0] * e.first.first, q[1] * e.first.second);
      int b = vid(q[0] * e.second.first, q[1] * e.second.second);
      dedges.insert({std::min(a, b), std::max(a, b)});
    }
  const int nE = (int)dedges.size();
  if (nV != n_vertices(d) || nE != n_diamond_edges(d))
    return fail(err, errlen, kTri, "diamond sizes differ from 2d^2+2d+1 / 6d^2+2d");
  std::vector<std::vector<int>> earlier(nV);
  for (auto& e : dedges) earlier[e.second].push_back(e.first);
  // antipodal boundary pairs (i,d-i)~(-i,i-d), (i,i-d)~(-i,d-i)
  std::set<std::pair<int, int>> pairs;
  for (int i = 0; i <= d; ++i) {
    int a = vid(i, d - i), b = vid(-i, i - d);
    pairs.insert({std::min(a, b), std::max(a, b)});
    a = vid(i, i - d);
    b = vid(-i, d - i);
    pairs.insert({std::min(a, b), std::max(a, b)});
  }
  const int nP = (int)pairs.size();
  if (nP != 2 * d) return fail(err, errlen, kTri, "expected 2d antipodal pairs");
  // --- program words ---
  prog->d = d;
  prog->nA = nA;
  prog->nV = nV;
  prog->nE = nE;
  prog->nP = nP;
  int off = 0;
  for (int v = 0; v < nV; ++v) {
    int x = vert[v].first, y = vert[v].second;
    int i = std::abs(x), j = std::abs(y);
    uint32_t p = (uint32_t)point_index(d, i, j);
    uint32_t g = (uint32_t)(((x < 0 ? i : 0) + (y < 0 ? j : 0)) & 1);
    std::sort(earlier[v].begin(), earlier[v].end());
    uint32_t n = (uint32_t)earlier[v].size();
    if (n > 255) return fail(err, errlen, kTri, "vertex degree too large");
    // the kernels use the first earlier neighbour as the spanning-tree parent
    if (v > 0 && n == 0) return fail(err, errlen, kTri, "a diamond vertex has no earlier neighbour");
    prog->words[v] = p | (g << 7) | (n << 8) | ((uint32_t)off << 16);
    for (int u : earlier[v]) prog->words[nV + off++] = (uint32_t)u;
  }
  int t = 0;
  for (auto& pr : pairs) prog->words[nV + nE + t++] = (uint32_t)pr.first | ((uint32_t)pr.second << 16);
  prog->n_words = nV + nE + nP;
  return 0;
}

int build_group_program(const HostProgram& full, int G, std::uint32_t* words, char* err, int errlen) {
  const int kArg = -1, kInternal = -5;
  const int d = full.d;
  if (G != 2 && G != 4) return fail(err, errlen, kArg, "lane group size must be 2 or 4");
  if (d < 2 || d > kDMax || !words) return fail(err, errlen, kArg, "bad degree or null pointer");
  // diamond vertices in program order (rows y = -d..d, x ascending)
  std::vector<Pt> vert;
  for (int y = -d; y <= d; ++y)
    for (int x = -d; x <= d; ++x)
      if (std::abs(x) + std::abs(y) <= d) vert.push_back({x, y});
  if ((int)vert.size() != full.nV) return fail(err, errlen, kInternal, "diamond size mismatch");
  // block 0: y >= 0 (and x >= 0 for G = 4), numbered in diamond order
  auto in_block0 = [&](Pt p) { return p.second >= 0 && (G == 2 || p.first >= 0); };
  std::vector<int> local(full.nV, -1);
  std::vector<int> of_local;
  for (int v = 0; v < full.nV; ++v)
    if (in_block0(vert[v])) {
      local[v] = (int)of_local.size();
      of_local.push_back(v);
    }
  const int NB = (int)of_local.size();
  if (NB != group_block_vertices(d, G)) return fail(err, errlen, kInternal, "block size mismatch");
  // records and earlier-neighbour lists (the diamond's, restricted to the block)
  int off = 0;
  std::vector<std::uint32_t> nbrs;
  for (int b = 0; b < NB; ++b) {
    const int v = of_local[b];
    const int x = vert[v].first, y = vert[v].second;
    const std::uint32_t rec = full.words[v];
    const std::uint32_t n_all = (rec >> 8) & 0xFF, off_all = rec >> 16;
    std::uint32_t n = 0;
    for (std::uint32_t k = 0; k < n_all; ++k) {
      const int u = (int)full.words[full.nV + off_all + k];
      if (local[u] >= 0) {
        // the neighbour's block id, with its lattice point and reflection
        // parity (bits 0..7 of its record) in bits 16..23
        nbrs.push_back((std::uint32_t)local[u] | ((full.words[u] & 0xFF) << 16));
        ++n;
      }
    }
    // the kernels take the first earlier neighbour as the spanning-tree parent
    if (b > 0 && n == 0) return fail(err, errlen, kInternal, "a block vertex has no earlier neighbour");
    if (off >= (1 << 12)) return fail(err, errlen, kInternal, "neighbour list too long");
    words[b] = (rec & 0xFF) | (n << 8) | ((std::uint32_t)off << 16) | ((std::uint32_t)(x == 0) << 28) |
               ((std::uint32_t)(y == 0) << 29);
    off += (int)n;
  }
  if (off != group_block_edges(d, G)) return fail(err, errlen, kInternal, "block edge count mismatch");
  for (int k = 0; k < off; ++k) words[NB + k] = nbrs[k];
  int at = NB + off;
  // glues, in the order the device derives its tree parents
  const int dx = 1, dy = G == 4 ? 2 : 1;
  int n_glue = 0;
  for (int q = 1; q < G; ++q) {
    const int sx = G == 4 ? (q & 1) : 0, sy = G == 4 ? (q >> 1) : q;
    for (int b = 0; b < NB; ++b) {
      const Pt p = vert[of_local[b]];
      const bool gx = sx && p.first == 0, gy = sy && p.second == 0;
      if (!gx && !gy) continue;
      const int partner = q - (gx ? dx : dy);
      words[at++] = (std::uint32_t)(b * G + partner) | ((std::uint32_t)(b * G + q) << 16);
      ++n_glue;
    }
  }
  if (n_glue != group_glues(d, G)) return fail(err, errlen, kInternal, "glue count mismatch");
  // antipodal pairs: each diamond point through the lowest block that holds it
  auto gidx = [&](int v) {
    const int x = vert[v].first, y = vert[v].second;
    const int sx = G == 4 && x < 0 ? 1 : 0, sy = y < 0 ? 1 : 0;
    const int q = G == 4 ? sx + 2 * sy : sy;
    const Pt p0{G == 4 ? std::abs(x) : x, std::abs(y)};
    int b = -1;
    for (int k = 0; k < NB; ++k)
      if (vert[of_local[k]] == p0) b = k;
    return b * G + q;
  };
  for (int t = 0; t < full.nP; ++t) {
    const std::uint32_t w = full.words[full.nV + full.nE + t];
    int a = gidx((int)(w & 0xFFFF)), b = gidx((int)(w >> 16));
    if (a > b) std::swap(a, b);
    words[at++] = (std::uint32_t)a | ((std::uint32_t)b << 16);
  }
  if (at != group_program_words(d, G)) return fail(err, errlen, kInternal, "group program size mismatch");
  return 0;
}

}  // namespace pw
