// search.hip -- the search over triangulations of Sec. 3, on the device:
//   * random flips of unimodular triangulations (an interior edge whose two
//     triangles form a parallelogram is replaced by the other diagonal),
//     plain or in pairs that keep the symmetry (i, j) -> (j, i);
//   * the reflected-diamond program of each triangulation (the layout the
//     scheme kernels walk, Alg. 1 first steps), built on the device;
//   * every triangulation of a batch judged against a pool of witness sign
//     distributions by the exact evaluation (the second search mode);
//   * per-triangulation objectives (distinct schemes, or schemes with a
//     target (p, n)) and the accept step of simulated annealing.
// A triangulation lives on the device as 64 adjacency rows (uint64): bit q
// of row p is set iff the lattice points p and q are joined by an edge
// (points numbered as in eq. (signs); |A| <= 64, so d <= 9).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "patchwork.h"
#include "pw_device.h"
#include "pw_host.h"

namespace pw {
namespace {

constexpr int kAdjRows = 64;
constexpr int kSearchMaxDegree = 9;
constexpr int kMaxNbr = 96;  // earlier neighbours of one diamond vertex (a program field holds 255)

// SplitMix64 finaliser used as a counter-based generator (Steele, Lea,
// Flood 2014): the draw for (walker w, counter c) is
// mix64(seed ^ mix64(w * 0x100000001B3 + c)).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t w, uint64_t c) {
  return mix64(seed ^ mix64(w * 0x100000001B3ull + c));
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ __forceinline__ int rdl(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// (i, j) of lattice point k of degree d (-1, -1 beyond |A|)
__device__ __forceinline__ void point_ij(int d, int k, int& i, int& j) {
  i = j = -1;
  int base = 0;
  for (int r = 0; r <= d; ++r) {
    const int w = d + 1 - r;
    if (k < base + w) {
      i = k - base;
      j = r;
      return;
    }
    base += w;
  }
}

__device__ __forceinline__ int point_idx(int d, int i, int j) { return j * (d + 1) - j * (j - 1) / 2 + i; }

// k-th set bit (k < popcount) of a wave-uniform mask
__device__ __forceinline__ int select_bit(uint64_t m, int k) {
  for (int t = 0; t < k; ++t) m &= m - 1;
  return __builtin_ctzll(m);
}

struct Flip {
  int a, b, c, e;  // edge ab, left apex c, right apex e
  bool ok;
};

// Can edge ab be flipped?  Its triangles are the unimodular ones over a
// common neighbour (det(b - a, c - a) = +1 left, -1 right); the flip is
// possible iff both exist and form a parallelogram (c + e = a + b: for two
// unimodular triangles a convex quadrilateral is a parallelogram).  All
// arguments and results are wave-uniform; the lane of point p holds
// row (its adjacency), pi, pj (its coordinates).
__device__ __forceinline__ Flip try_flip(uint64_t row, int pi, int pj, int a, int b) {
  Flip f{a, b, -1, -1, false};
  const uint64_t ra = readlane64(row, a), rb = readlane64(row, b);
  if (!((ra >> b) & 1)) return f;
  const int ia = rdl(pi, a), ja = rdl(pj, a), ib = rdl(pi, b), jb = rdl(pj, b);
  const int vx = ib - ia, vy = jb - ja;
  uint64_t common = ra & rb;
  while (common) {
    const int c = __builtin_ctzll(common);
    common &= common - 1;
    const int det = vx * (rdl(pj, c) - ja) - vy * (rdl(pi, c) - ia);
    if (det == 1) f.c = c;
    if (det == -1) f.e = c;
  }
  if (f.c < 0 || f.e < 0) return f;
  f.ok = rdl(pi, f.c) + rdl(pi, f.e) == ia + ib && rdl(pj, f.c) + rdl(pj, f.e) == ja + jb;
  return f;
}

__device__ __forceinline__ void apply_flip(uint64_t& row, int lane, const Flip& f) {
  if (lane == f.a) row &= ~(1ull << f.b);
  if (lane == f.b) row &= ~(1ull << f.a);
  if (lane == f.c) row |= 1ull << f.e;
  if (lane == f.e) row |= 1ull << f.c;
}

__device__ __forceinline__ bool same_edge(int a, int b, int x, int y) { return (a == x && b == y) || (a == y && b == x); }

// One wave per triangulation; `steps` proposed moves each.  Move s draws
// r1 = draw(seed, w, 2 (step0 + s)), r2 = draw(seed, w, 2 (step0 + s) + 1):
// a = r1 mod |A|, b = the (r2 mod deg a)-th neighbour of a in increasing
// point order; the edge ab is flipped if it can be.  Symmetric mode, with
// s(i, j) = (j, i): if s maps ab to itself the flip alone keeps the
// symmetry; otherwise ab and s(ab) are flipped together when both can be
// and their quadrilaterals share no triangle (then the two flips commute and
// the pair is s-invariant); other moves leave T unchanged.
__global__ __launch_bounds__(256) void k_flip_walk(int d, uint64_t* __restrict__ adj, int64_t n, int steps,
                                                   int symmetric, uint64_t seed, uint64_t step0,
                                                   uint32_t* __restrict__ moves) {
  const int lane = threadIdx.x & 63;
  const int nA = n_points(d);
  int pi, pj;
  point_ij(d, lane, pi, pj);
  const int sw = lane < nA ? point_idx(d, pj, pi) : lane;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_id(); w < n; w += waves) {
    uint64_t row = lane < nA ? adj[w * kAdjRows + lane] : 0;
    uint32_t done = 0;
    for (int s = 0; s < steps; ++s) {
      const uint64_t ctr = 2 * (step0 + (uint64_t)s);
      const uint64_t r1 = draw(seed, (uint64_t)w, ctr), r2 = draw(seed, (uint64_t)w, ctr + 1);
      const int a = (int)(r1 % (uint64_t)nA);
      const uint64_t ra = readlane64(row, a);
      const int deg = __builtin_popcountll(ra);
      if (deg == 0) continue;
      const int b = select_bit(ra, (int)(r2 % (uint64_t)deg));
      const Flip f = try_flip(row, pi, pj, a, b);
      if (!f.ok) continue;
      if (!symmetric) {
        apply_flip(row, lane, f);
        ++done;
        continue;
      }
      const int sa = rdl(sw, a), sb = rdl(sw, b);
      if (same_edge(a, b, sa, sb)) {
        apply_flip(row, lane, f);
        ++done;
        continue;
      }
      const Flip g = try_flip(row, pi, pj, sa, sb);
      if (!g.ok) continue;
      // a shared triangle would make s(ab) a side of ab's quadrilateral
      if (same_edge(sa, sb, a, f.c) || same_edge(sa, sb, b, f.c) || same_edge(sa, sb, a, f.e) ||
          same_edge(sa, sb, b, f.e))
        continue;
      apply_flip(row, lane, f);
      apply_flip(row, lane, g);
      ++done;
    }
    if (lane < nA) adj[w * kAdjRows + lane] = row;
    if (moves && lane == 0) moves[w] += done;
  }
}

// ------------------------------------------------------------ programs

// Diamond rows y = -d..d, x ascending: index of the first vertex of row y
__device__ __forceinline__ int row_start(int d, int y) {
  return y <= 0 ? (y + d) * (y + d) : d * d + y * (2 * d + 1) - y * (y - 1);
}
__device__ __forceinline__ int vid(int d, int x, int y) {
  const int ay = y < 0 ? -y : y;
  return row_start(d, y) + x + (d - ay);
}

// visit the diamond neighbours of vertex (x, y): the reflections (ex iq,
// ey jq) of the triangulation's neighbours q of (|x|, |y|), ex over the
// signs that map |x| to x (both when x = 0, but once when iq = 0 too, as
// both give the same vertex), ey likewise
template <class F>
__device__ __forceinline__ void for_each_nbr(int d, int x, int y, uint64_t rowp, const int8_t* pti,
                                             const int8_t* ptj, F&& f) {
  while (rowp) {
    const int q = __builtin_ctzll(rowp);
    rowp &= rowp - 1;
    const int iq = pti[q], jq = ptj[q];
    for (int sx = -1; sx <= 1; sx += 2) {
      if (x != 0 && (sx < 0) != (x < 0)) continue;
      if (iq == 0 && x == 0 && sx < 0) continue;  // (0, .) once
      for (int sy = -1; sy <= 1; sy += 2) {
        if (y != 0 && (sy < 0) != (y < 0)) continue;
        if (jq == 0 && y == 0 && sy < 0) continue;
        f(vid(d, sx * iq, sy * jq));
      }
    }
  }
}

// One wave per triangulation: the program of tri.cpp's build_program
// (vertex records p | g << 7 | n << 8 | off << 16, the earlier neighbours of
// each vertex in increasing order, the 2d antipodal pairs a | b << 16 in
// increasing (a, b) order).  bad[t] != 0 marks a triangulation whose
// program could not be built (a vertex without or with too many earlier
// neighbours, or a diamond edge count other than 6d^2 + 2d).
__global__ __launch_bounds__(64) void k_build_programs(int d, const uint64_t* __restrict__ adj, int64_t n,
                                                       uint32_t* __restrict__ progs, int prog_words,
                                                       uint32_t* __restrict__ bad) {
  __shared__ uint64_t rows[kAdjRows];
  __shared__ int8_t pti[kAdjRows], ptj[kAdjRows];
  const int lane = threadIdx.x;
  const int nA = n_points(d), nV = n_vertices(d), nE = n_diamond_edges(d);
  {
    int i, j;
    point_ij(d, lane, i, j);
    pti[lane] = (int8_t)i;
    ptj[lane] = (int8_t)j;
  }
  for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
    __syncthreads();
    rows[lane] = lane < nA ? adj[t * kAdjRows + lane] : 0;
    __syncthreads();
    uint32_t* prog = progs + t * (int64_t)prog_words;
    uint32_t err = 0;
    int base = 0;  // earlier-neighbour entries of the vertices before this round
    for (int v0 = 0; v0 < nV; v0 += 64) {
      const int v = v0 + lane;
      int x = 0, y = -d;
      if (v < nV) {
        while (y < d && row_start(d, y + 1) <= v) ++y;
        const int ay = y < 0 ? -y : y;
        x = v - row_start(d, y) - (d - ay);
      }
      const int ax = x < 0 ? -x : x, ay = y < 0 ? -y : y;
      const int p = v < nV ? point_idx(d, ax, ay) : 0;
      const uint64_t rowp = v < nV ? rows[p] : 0;
      int cnt = 0;
      for_each_nbr(d, x, y, rowp, pti, ptj, [&](int u) { cnt += u < v; });
      if (v < nV && (cnt > kMaxNbr || (v > 0 && cnt == 0))) err = 1;
      // exclusive prefix over the round's lanes
      int incl = cnt;
      for (int o = 1; o < 64; o <<= 1) {
        const int up = __shfl_up(incl, o);
        if (lane >= o) incl += up;
      }
      const int off = base + incl - cnt;
      base += __shfl(incl, 63);
      if (v < nV) {
        const uint32_t g = (uint32_t)(((x < 0 ? ax : 0) + (y < 0 ? ay : 0)) & 1);
        prog[v] = (uint32_t)p | (g << 7) | ((uint32_t)(cnt & 0xFF) << 8) | ((uint32_t)off << 16);
        // each earlier neighbour goes to its rank among them
        if (off + cnt <= nE && cnt <= kMaxNbr) {
          for_each_nbr(d, x, y, rowp, pti, ptj, [&](int u) {
            if (u >= v) return;
            int rank = 0;
            for_each_nbr(d, x, y, rowp, pti, ptj, [&](int u2) { rank += u2 < u; });
            prog[nV + off + rank] = (uint32_t)u;
          });
        }
      }
    }
    if (base != nE) err = 1;
    // antipodal pairs: (i, d-i) ~ (-i, i-d) and (i, i-d) ~ (-i, d-i); the
    // corner pairs occur in both families and are kept once
    const int np = 2 * (d + 1);
    uint32_t key = 0xFFFFFFFFu;
    if (lane < np) {
      const int i = lane % (d + 1);
      int a, b;
      if (lane <= d) {
        a = vid(d, i, d - i);
        b = vid(d, -i, i - d);
      } else {
        a = vid(d, i, i - d);
        b = vid(d, -i, d - i);
      }
      if (b < a) {
        const int tmp = a;
        a = b;
        b = tmp;
      }
      key = ((uint32_t)a << 16) | (uint32_t)b;
    }
    int rank = 0;
    bool first = true;
    for (int l = 0; l < np; ++l) {
      const uint32_t k2 = (uint32_t)__shfl((int)key, l);
      rank += k2 < key;
      if (k2 == key && l < lane) first = false;
    }
    // duplicates counted once: the rank among distinct keys
    int dup_below = 0;
    for (int l = 0; l < np; ++l) {
      const uint32_t k2 = (uint32_t)__shfl((int)key, l);
      bool k2_first = true;
      for (int m = 0; m < l; ++m)
        if ((uint32_t)__shfl((int)key, m) == k2) k2_first = false;
      dup_below += (k2 < key && !k2_first);
    }
    if (lane < np && first) {
      const int r = rank - dup_below;
      if (r < 2 * d) prog[nV + nE + r] = (key >> 16) | ((key & 0xFFFFu) << 16);
    }
    // a program that could not be built keeps no neighbour lists (every
    // count and offset 0, every listed neighbour vertex 0), so that an
    // evaluation of it reads only its own words and in-range vertices (and
    // fails its checks)
    const bool any_err = __ballot(err != 0) != 0;
    if (any_err) {
      __syncthreads();
      for (int v = lane; v < nV; v += 64) prog[v] &= 0xFFu;
      for (int k = lane; k < nE; k += 64) prog[nV + k] = 0;
    }
    if (lane == 0) bad[t] = any_err ? 1u : 0u;
  }
}

// --------------------------------------------------------- evaluation

// Every triangulation of the batch against every witness: one wave takes
// 64 witnesses of one triangulation at a time; code index t * n_w + w.
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Cfg<D>::WAVES_PER_EU))) void k_programs(
    const uint32_t* __restrict__ progs, int prog_words, int64_t n_tris, const uint64_t* __restrict__ masks,
    int64_t n_w, uint64_t* __restrict__ codes, const HistDev* __restrict__ h, uint32_t* __restrict__ errflag) {
  using C = Cfg<D>;
  extern __shared__ uint32_t smem[];
  __shared__ uint8_t par_rows[C::WAVES * C::PAR_ROWS * 64];
  const Lane L = lane_memory_split<D>(smem, par_rows);
  const int lane = threadIdx.x & 63;
  const int64_t per_tri = (n_w + 63) / 64;
  const int64_t items = n_tris * per_tri;
  const int64_t waves = (int64_t)gridDim.x * C::WAVES;
  WaveTable tab;
  tab.clear();
  uint32_t errs = 0;
  for (int64_t it = (int64_t)blockIdx.x * C::WAVES + wave_id(); it < items; it += waves) {
    const int64_t t = it / per_tri;
    const int64_t w = (it - t * per_tri) * 64 + lane;
    const bool valid = w < n_w;
    const uint32_t* prog = progs + t * (int64_t)prog_words;
    typename C::Mask m = 0;
    if (valid) {
      if constexpr (sizeof(typename C::Mask) == 8) {
        m = masks[2 * w];
      } else {
        m = ((u128)masks[2 * w + 1] << 64) | (u128)masks[2 * w];
      }
    }
    const u128 code = Eval<D>::run(prog, m, L, errs);
    const int64_t gi = t * n_w + w;
    if (codes && valid) store_code(codes, gi, code);
    if (h) tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, (uint64_t)gi, lane, h);
  }
  if (h) tab.flush(h);
  if (errs) atomicOr(errflag, errs);
}

// ---------------------------------------------------------- objectives

// number of ovals at odd depth (p: outermost = depth 1) and at even depth
// (n) of a code whose bits fit in the low word (d <= 9: at most 2M + 1 <= 59)
__device__ __forceinline__ void code_pn(uint64_t lo, int& p, int& n) {
  p = n = 0;
  const int len = 64 - __builtin_clzll(lo);
  int depth = 0;
  for (int k = len - 2; k >= 0; --k) {
    if ((lo >> k) & 1) {
      ++depth;
      if (depth & 1) ++p;
      else ++n;
    } else {
      --depth;
    }
  }
}

// true iff lo is in the sorted list known[0 .. n_known)
__device__ __forceinline__ bool in_sorted(const uint64_t* __restrict__ known, int n_known, uint64_t lo) {
  int a = 0, b = n_known;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (known[m] < lo) a = m + 1;
    else b = m;
  }
  return a < n_known && known[a] == lo;
}

// One wave per triangulation over its n_w codes (t * n_w .. + n_w - 1):
// mode 0 = number of distinct codes (an open-addressing set in LDS of
// `cap` slots, cap a power of two >= 2 n_w); mode 1 = number of codes
// with (p, n) = (tp, tn); mode 2 = number of distinct codes not in the
// sorted list `known` (the types a triangulation adds to those found).
// Failed evaluations (code 0) count for nothing.
__global__ __launch_bounds__(64) void k_objective(const uint64_t* __restrict__ codes, int64_t n_tris, int n_w,
                                                  int mode, int tp, int tn, const uint64_t* __restrict__ known,
                                                  int n_known, int cap, float* __restrict__ score) {
  extern __shared__ uint64_t slots[];
  const int lane = threadIdx.x;
  for (int64_t t = blockIdx.x; t < n_tris; t += gridDim.x) {
    int count = 0;
    if (mode != 1) {
      for (int s = lane; s < cap; s += 64) slots[s] = 0;
      __syncthreads();
      for (int w = lane; w < n_w; w += 64) {
        const uint64_t lo = codes[2 * (t * n_w + w)];
        if (lo == 0) continue;
        if (mode == 2 && in_sorted(known, n_known, lo)) continue;
        uint32_t s = (uint32_t)((lo * 0x9E3779B97F4A7C15ull) >> 40) & (uint32_t)(cap - 1);
        while (true) {
          const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&slots[s]), 0ull,
                                                   (unsigned long long)lo);
          if (old == 0) {
            ++count;
            break;
          }
          if (old == lo) break;
          s = (s + 1) & (uint32_t)(cap - 1);
        }
      }
      __syncthreads();
    } else {
      for (int w = lane; w < n_w; w += 64) {
        const uint64_t lo = codes[2 * (t * n_w + w)];
        if (lo == 0) continue;
        int p, n;
        code_pn(lo, p, n);
        count += (p == tp && n == tn);
      }
    }
    for (int o = 32; o > 0; o >>= 1) count += __shfl_down(count, o);
    if (lane == 0) score[t] = (float)count;
  }
}

// Metropolis step of simulated annealing (maximising the score), one wave
// per chain: the proposal is accepted if it scores at least as high, or
// else if u < accept[k - 1] where k = score_cur - score_prop (a whole
// number) and u is the top 24 bits of draw(seed, chain, step); accept[]
// holds floor(2^24 exp(-k / temperature)) for k = 1 .. n_accept (0 beyond),
// computed by the caller, so the decision is exact integer arithmetic.
// Accepted: cur <- prop; rejected: prop <- cur.  best keeps the highest-
// scoring state a chain has held.
__global__ __launch_bounds__(64) void k_anneal_accept(uint64_t* __restrict__ cur, uint64_t* __restrict__ prop,
                                                      float* __restrict__ score_cur,
                                                      const float* __restrict__ score_prop,
                                                      uint64_t* __restrict__ best, float* __restrict__ score_best,
                                                      int64_t n, const uint32_t* __restrict__ accept, int n_accept,
                                                      uint64_t seed, uint64_t step, uint32_t* __restrict__ n_acc) {
  const int lane = threadIdx.x;
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const float sc = score_cur[w], sp = score_prop[w];
    bool take = sp >= sc;
    if (!take) {
      const int k = (int)(sc - sp);
      const uint32_t u = (uint32_t)(draw(seed, (uint64_t)w, step) >> 40);
      take = k >= 1 && k <= n_accept && u < accept[k - 1];
    }
    const uint64_t rc = cur[w * kAdjRows + lane], rp = prop[w * kAdjRows + lane];
    const uint64_t now = take ? rp : rc;
    cur[w * kAdjRows + lane] = now;
    prop[w * kAdjRows + lane] = now;
    const float s_now = take ? sp : sc;
    if (s_now > score_best[w]) {
      best[w * kAdjRows + lane] = now;
      __syncthreads();
      if (lane == 0) score_best[w] = s_now;
    }
    if (lane == 0) {
      score_cur[w] = s_now;
      if (take) n_acc[w] += 1;
    }
    __syncthreads();
  }
}

int prog_words_for(int d) { return n_vertices(d) + n_diamond_edges(d) + 2 * d; }

template <int D>
pw_status launch_programs(const uint32_t* progs, int64_t n_tris, const uint64_t* masks, int64_t n_w, uint64_t* codes,
                          const pw_hist* h, uint32_t* err, hipStream_t s) {
  using C = Cfg<D>;
  const size_t lds = (size_t)C::DYN_WORDS * 4 * 64 * C::WAVES;
  static const hipError_t attr =
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_programs<D>), hipFuncAttributeMaxDynamicSharedMemorySize,
                          160 * 1024 - C::WAVES * C::PAR_ROWS * 64);
  if (attr != hipSuccess) {
    (void)hipGetLastError();
    return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
  }
  const int64_t items = n_tris * ((n_w + 63) / 64);
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / ((int64_t)C::LANE_WORDS * 256 * C::WAVES)));
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((items + C::WAVES - 1) / C::WAVES, cu_count() * per_cu));
  hipLaunchKernelGGL(k_programs<D>, dim3((unsigned)blocks), dim3(64 * C::WAVES), lds, s, progs, prog_words_for(D),
                     n_tris, masks, n_w, codes, h ? h->d_dev : nullptr, err);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

}  // namespace
}  // namespace pw

using namespace pw;

extern "C" {

int32_t pw_program_words(int32_t d) {
  if (d < 1 || d > kDMax) return PW_ERR_ARG;
  return prog_words_for(d);
}

pw_status pw_adjacency_from_edges(int32_t d, const int16_t* edges_ij, int32_t n_edges, uint64_t* rows) {
  if (d < 1 || d > kSearchMaxDegree || !rows) return set_err(PW_ERR_ARG, "degree %d (1..9) or null rows", d);
  HostProgram prog;
  char msg[256];
  const int rc = build_program(d, edges_ij, n_edges, &prog, msg, sizeof msg);
  if (rc != 0) return set_err(rc, "%s", msg);
  std::memset(rows, 0, sizeof(uint64_t) * kAdjRows);
  auto idx = [d](int i, int j) { return j * (d + 1) - j * (j - 1) / 2 + i; };
  for (int e = 0; e < n_edges; ++e) {
    const int p = idx(edges_ij[4 * e], edges_ij[4 * e + 1]), q = idx(edges_ij[4 * e + 2], edges_ij[4 * e + 3]);
    rows[p] |= 1ull << q;
    rows[q] |= 1ull << p;
  }
  return PW_OK;
}

pw_status pw_edges_from_adjacency(int32_t d, const uint64_t* rows, int16_t* edges_ij, int32_t cap, int32_t* n_edges) {
  if (d < 1 || d > kSearchMaxDegree || !rows) return set_err(PW_ERR_ARG, "degree %d (1..9) or null rows", d);
  std::vector<std::pair<int, int>> pts;
  for (int j = 0; j <= d; ++j)
    for (int i = 0; i + j <= d; ++i) pts.push_back({i, j});
  const int nA = (int)pts.size();
  int n = 0;
  for (int p = 0; p < nA; ++p)
    for (int q = p + 1; q < nA; ++q) {
      if (!((rows[p] >> q) & 1)) continue;
      if (((rows[q] >> p) & 1) == 0) return set_err(PW_ERR_TRI, "adjacency is not symmetric at (%d, %d)", p, q);
      if (edges_ij && n < cap) {
        edges_ij[4 * n] = (int16_t)pts[p].first;
        edges_ij[4 * n + 1] = (int16_t)pts[p].second;
        edges_ij[4 * n + 2] = (int16_t)pts[q].first;
        edges_ij[4 * n + 3] = (int16_t)pts[q].second;
      }
      ++n;
    }
  for (int p = nA; p < kAdjRows; ++p)
    if (rows[p]) return set_err(PW_ERR_TRI, "row %d beyond |A| is not empty", p);
  if (n_edges) *n_edges = n;
  if (edges_ij && n > cap) return set_err(PW_ERR_ARG, "%d edges, buffer holds %d", n, cap);
  return PW_OK;
}

pw_status pw_flip_walk(int32_t d, uint64_t* d_adj, int64_t n_tris, int32_t steps, int32_t symmetric, uint64_t seed,
                       uint64_t step0, uint32_t* d_moves, hipStream_t stream) {
  if (d < 1 || d > kSearchMaxDegree || n_tris < 0 || steps < 0 || (n_tris > 0 && !d_adj))
    return set_err(PW_ERR_ARG, "bad flip walk arguments (d %d, n %lld, steps %d)", d, (long long)n_tris, steps);
  if (n_tris == 0 || steps == 0) return PW_OK;
  const int64_t blocks = std::min<int64_t>((n_tris + 3) / 4, (int64_t)cu_count() * 8);
  hipLaunchKernelGGL(k_flip_walk, dim3((unsigned)blocks), dim3(256), 0, stream, d, d_adj, n_tris, steps, symmetric,
                     seed, step0, d_moves);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_build_programs(int32_t d, const uint64_t* d_adj, int64_t n_tris, uint32_t* d_progs, uint32_t* d_bad,
                            hipStream_t stream) {
  if (d < 1 || d > kSearchMaxDegree || n_tris < 0 || (n_tris > 0 && (!d_adj || !d_progs || !d_bad)))
    return set_err(PW_ERR_ARG, "bad program build arguments (d %d, n %lld)", d, (long long)n_tris);
  if (n_tris == 0) return PW_OK;
  const int64_t blocks = std::min<int64_t>(n_tris, (int64_t)cu_count() * 16);
  hipLaunchKernelGGL(k_build_programs, dim3((unsigned)blocks), dim3(64), 0, stream, d, d_adj, n_tris, d_progs,
                     prog_words_for(d), d_bad);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status patchwork_scheme_programs(int32_t d, const uint32_t* d_progs, int64_t n_tris, const uint64_t* d_masks,
                                    int64_t n_w, uint64_t* d_codes, pw_hist_t hist, uint32_t* d_err,
                                    hipStream_t stream) {
  if (d < 1 || d > kDMax || n_tris < 0 || n_w < 0) return set_err(PW_ERR_ARG, "bad degree or sizes");
  if (n_tris == 0 || n_w == 0) return PW_OK;
  if (!d_progs || !d_masks || !d_err || (!d_codes && !hist)) return set_err(PW_ERR_ARG, "null buffer");
  if ((uintptr_t)d_codes & 15) return set_err(PW_ERR_ARG, "d_codes must be 16-byte aligned");
  switch (d) {
    case 1: return launch_programs<1>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 2: return launch_programs<2>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 3: return launch_programs<3>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 4: return launch_programs<4>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 5: return launch_programs<5>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 6: return launch_programs<6>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 7: return launch_programs<7>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 8: return launch_programs<8>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 9: return launch_programs<9>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 10: return launch_programs<10>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 11: return launch_programs<11>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    case 12: return launch_programs<12>(d_progs, n_tris, d_masks, n_w, d_codes, hist, d_err, stream);
    default: return set_err(PW_ERR_ARG, "degree %d", d);
  }
}

pw_status pw_tri_objective(int32_t d, const uint64_t* d_codes, int64_t n_tris, int32_t n_w, int32_t mode,
                           int32_t target_p, int32_t target_n, const uint64_t* d_known, int32_t n_known,
                           float* d_score, hipStream_t stream) {
  if (d < 1 || d > kSearchMaxDegree || n_tris < 0 || n_w < 0 || n_w > 8192 || mode < 0 || mode > 2 ||
      n_known < 0)
    return set_err(PW_ERR_ARG, "bad objective arguments (d %d, n_w %d, mode %d)", d, n_w, mode);
  if (n_tris == 0) return PW_OK;
  if (!d_codes || !d_score || (mode == 2 && n_known > 0 && !d_known)) return set_err(PW_ERR_ARG, "null buffer");
  int cap = 64;
  while (cap < 2 * n_w) cap <<= 1;
  const size_t lds = mode != 1 ? sizeof(uint64_t) * cap : 0;
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_objective),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (attr != hipSuccess) {
    (void)hipGetLastError();
    return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
  }
  const int64_t blocks = std::min<int64_t>(n_tris, (int64_t)cu_count() * 8);
  hipLaunchKernelGGL(k_objective, dim3((unsigned)blocks), dim3(64), lds, stream, d_codes, n_tris, n_w, mode, target_p,
                     target_n, d_known, mode == 2 ? n_known : 0, cap, d_score);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

pw_status pw_anneal_accept(uint64_t* d_cur, uint64_t* d_prop, float* d_score_cur, const float* d_score_prop,
                           uint64_t* d_best, float* d_score_best, int64_t n_chains, const uint32_t* d_accept,
                           int32_t n_accept, uint64_t seed, uint64_t step, uint32_t* d_n_accepted,
                           hipStream_t stream) {
  if (n_chains < 0 || n_accept < 0) return set_err(PW_ERR_ARG, "negative size");
  if (n_chains == 0) return PW_OK;
  if (!d_cur || !d_prop || !d_score_cur || !d_score_prop || !d_best || !d_score_best || !d_n_accepted ||
      (n_accept > 0 && !d_accept))
    return set_err(PW_ERR_ARG, "null buffer");
  const int64_t blocks = std::min<int64_t>(n_chains, (int64_t)cu_count() * 16);
  hipLaunchKernelGGL(k_anneal_accept, dim3((unsigned)blocks), dim3(64), 0, stream, d_cur, d_prop, d_score_cur,
                     d_score_prop, d_best, d_score_best, n_chains, d_accept, n_accept, seed, step, d_n_accepted);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

}  // extern "C"
