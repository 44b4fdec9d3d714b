// sym.cpp -- the symmetries that reduce the search space (Sec. 3, Table 1):
// the S3 action on triangulations of d*Delta_2 by permutations of the
// barycentric coordinates (i, j, d-i-j), and the choice of (Z/2)^3 class
// representatives of sign distributions.  Host code only; nothing here
// touches the device.
#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "patchwork.h"
#include "pw_internal.h"

namespace pw {
__attribute__((format(printf, 2, 3))) pw_status set_err(pw_status code, const char* fmt, ...);
}

using namespace pw;

namespace {

// The six permutations of the barycentric coordinates, in lexicographic
// order; permutation k sends (i, j) to (b[P[0]], b[P[1]]) with
// b = (i, j, d - i - j).
constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

inline int point_index(int d, int i, int j) { return j * (d + 1) - j * (j - 1) / 2 + i; }

inline void image(int d, int k, int i, int j, int& oi, int& oj) {
  const int b[3] = {i, j, d - i - j};
  oi = b[kPerm[k][0]];
  oj = b[kPerm[k][1]];
}

using Edge = std::array<int16_t, 4>;  // (i0, j0, i1, j1), endpoint with the smaller point index first

// The edge list of permutation k applied to `edges`, each edge written with
// its endpoints in point-index order and the list sorted.
std::vector<Edge> permuted(int d, int k, const int16_t* edges, int n) {
  std::vector<Edge> out(n);
  for (int e = 0; e < n; ++e) {
    int a0, a1, b0, b1;
    image(d, k, edges[4 * e], edges[4 * e + 1], a0, a1);
    image(d, k, edges[4 * e + 2], edges[4 * e + 3], b0, b1);
    if (point_index(d, b0, b1) < point_index(d, a0, a1)) {
      std::swap(a0, b0);
      std::swap(a1, b1);
    }
    out[e] = Edge{(int16_t)a0, (int16_t)a1, (int16_t)b0, (int16_t)b1};
  }
  std::sort(out.begin(), out.end(), [d](const Edge& x, const Edge& y) {
    const int x0 = point_index(d, x[0], x[1]), y0 = point_index(d, y[0], y[1]);
    if (x0 != y0) return x0 < y0;
    return point_index(d, x[2], x[3]) < point_index(d, y[2], y[3]);
  });
  return out;
}

bool less_list(int d, const std::vector<Edge>& x, const std::vector<Edge>& y) {
  for (size_t e = 0; e < x.size(); ++e) {
    for (int c = 0; c < 4; c += 2) {
      const int px = point_index(d, x[e][c], x[e][c + 1]), py = point_index(d, y[e][c], y[e][c + 1]);
      if (px != py) return px < py;
    }
  }
  return false;
}

}  // namespace

extern "C" {

pw_status pw_tri_canonical(int32_t d, const int16_t* edges_ij, int32_t n_edges, int16_t* out_edges,
                           int32_t* perm_index, int32_t* stabilizer) {
  HostProgram prog;
  char msg[256];
  const int rc = build_program(d, edges_ij, n_edges, &prog, msg, sizeof msg);
  if (rc != 0) return set_err(rc, "%s", msg);
  std::vector<Edge> best = permuted(d, 0, edges_ij, n_edges), self = best;
  int best_k = 0, stab = 1;
  for (int k = 1; k < 6; ++k) {
    const std::vector<Edge> img = permuted(d, k, edges_ij, n_edges);
    if (img == self) ++stab;
    if (less_list(d, img, best)) {
      best = img;
      best_k = k;
    }
  }
  if (out_edges)
    for (int e = 0; e < n_edges; ++e)
      for (int c = 0; c < 4; ++c) out_edges[4 * e + c] = best[e][c];
  if (perm_index) *perm_index = best_k;
  if (stabilizer) *stabilizer = stab;
  return PW_OK;
}

pw_status pw_point_map(int32_t d, int32_t perm_index, int32_t* out) {
  if (d < 1 || d > kDMax || perm_index < 0 || perm_index > 5 || !out)
    return set_err(PW_ERR_ARG, "bad degree %d, permutation %d or null output", d, perm_index);
  for (int j = 0; j <= d; ++j)
    for (int i = 0; i + j <= d; ++i) {
      int a, b;
      image(d, perm_index, i, j, a, b);
      out[point_index(d, i, j)] = point_index(d, a, b);
    }
  return PW_OK;
}

pw_status pw_class_fixed_bits(int32_t d, uint64_t out[2]) {
  if (d < 1 || d > kDMax || !out) return set_err(PW_ERR_ARG, "bad degree %d or null output", d);
  if (d < 2) return set_err(PW_ERR_ARG, "d = 1 has no three points of distinct parity classes");
  const int nA = n_points(d);
  // (0,0), then two points of two distinct nonzero parity classes
  // (i mod 2, j mod 2); three distinct classes make the
  // vectors (1, i, j) independent mod 2, so every (Z/2)^3 orbit has exactly
  // one member that is '+' on the three.  Points from index 10 on are
  // preferred, leaving lattice points 1..9 free.
  int chosen[2] = {-1, -1}, cls[2] = {-1, -1};
  for (int start : {10, 1}) {
    chosen[0] = chosen[1] = cls[0] = cls[1] = -1;
    int got = 0;
    for (int j = 0; j <= d && got < 2; ++j)
      for (int i = 0; i + j <= d && got < 2; ++i) {
        const int k = point_index(d, i, j);
        const int c = (i & 1) | ((j & 1) << 1);
        if (k < start || c == 0 || c == cls[0]) continue;
        chosen[got] = k;
        cls[got] = c;
        ++got;
      }
    if (got == 2) break;
  }
  if (chosen[1] < 0 || chosen[1] >= nA) return set_err(PW_ERR_ARG, "no class representatives for d = %d", d);
  out[0] = out[1] = 0;
  for (int k : {0, chosen[0], chosen[1]}) out[k / 64] |= 1ull << (k % 64);
  return PW_OK;
}

}  // extern "C"
