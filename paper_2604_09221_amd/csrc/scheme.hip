// scheme.hip -- gfx950 kernels for Algorithm 1 ("Fast Isotopy Computation
// for T-Curves", Sec. 2): one sign mask per lane, the triangulation program
// read with wave-uniform loads, per-lane union-find state in LDS.
//
// LDS layout: each wave owns LANE_WORDS * 64 dwords; word k of lane l sits
// at index k * 64 + l, so every lane always hits its own bank whatever the
// per-lane index (conflict-free for uniform and divergent accesses alike).
//
// Per mask (thread) the phases are:
//   1 components  (Alg. 1 "compute connected components of same-sign
//     vertices"): vertices in program order; each earlier neighbour with
//     the same sign is unioned.  Entry of v (u16): bits 0..8 parent,
//     bit 9 parity to parent, bit 10 odd-cycle flag (roots), bit 15 sign.
//     Links always go from the larger root to the smaller one, so every
//     parent index is smaller than its child's.
//   2 regions (Alg. 1 "coarsen into regions by identifying antipodal
//     boundary pairs"): union along the 2d pairs.  For even d the union
//     carries parity 1 (each identification reverses orientation, proof of
//     Thm. 2) and a same-parity closure marks an odd cycle.
//   3 region ids + adjacency (Alg. 1 "build region adjacency graph from
//     crossed edges"): vertices in order again; a root gets the next id, any
//     other vertex copies the id of its parent (already relabelled because
//     parents are smaller).  Crossed earlier edges add adjacency bits; a
//     crossed edge inside one region is the self-loop that marks the root
//     for odd d.
//   4 root, breadth-first order from the root and the canonical code
//     (Alg. 1, last step, AHU encoding): children codes sorted descending
//     by their left-aligned bit strings; leaves ('10') sort last.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "patchwork.h"
#include "pw_internal.h"

namespace pw {

typedef unsigned __int128 u128;

// ------------------------------------------------------------------ config

template <int D>
struct Cfg {
  static constexpr int NA = n_points(D);
  static constexpr int NV = n_vertices(D);
  static constexpr int NE = n_diamond_edges(D);
  static constexpr int NP = 2 * D;
  static constexpr int RMAX = harnack(D) + 1;  // regions = ovals + 1 <= M + 1
  static constexpr bool EVEN = (D % 2) == 0;
  using Mask = typename std::conditional<(NA <= 64), uint64_t, u128>::type;
  using Adj = typename std::conditional<(RMAX <= 32), uint32_t, uint64_t>::type;
  using Code = typename std::conditional<(D <= 9), uint64_t, u128>::type;
  static constexpr int ADJ_W = sizeof(Adj) / 4;
  static constexpr int CODE_W = sizeof(Code) / 4;
  static constexpr int E_WORDS = (NV + 1) / 2;
  // after phase 3 the entry words are reused for codes and order/parent
  static constexpr int TAIL_WORDS = RMAX * (CODE_W + 1);
  static constexpr int LOW_WORDS = E_WORDS > TAIL_WORDS ? E_WORDS : TAIL_WORDS;
  static constexpr int ADJ_BASE = LOW_WORDS;
  static constexpr int LANE_WORDS = LOW_WORDS + RMAX * ADJ_W;
  static constexpr int CODE_BASE = 0;
  static constexpr int ORD_BASE = RMAX * CODE_W;
  // waves per block: keep a block's LDS at or below 80 KiB
  static constexpr int WAVE_BYTES = LANE_WORDS * 4 * 64;
  static constexpr int WAVES = WAVE_BYTES * 4 <= 80 * 1024 ? 4 : (WAVE_BYTES * 2 <= 80 * 1024 ? 2 : 1);
};

// ------------------------------------------------------------ lane memory

struct Lane {
  uint32_t* w;  // word 0 of this lane; word k at w[k * 64]
  __device__ __forceinline__ uint32_t& word(int k) const { return w[k * 64]; }
  __device__ __forceinline__ uint16_t& ent(int v) const {
    return reinterpret_cast<uint16_t*>(w + (v >> 1) * 64)[v & 1];
  }
  __device__ __forceinline__ uint8_t& byte(int k, int b) const {
    return reinterpret_cast<uint8_t*>(w + k * 64)[b];
  }
};

constexpr uint32_t kParent = 0x1FFu;
constexpr uint32_t kParity = 1u << 9;
constexpr uint32_t kOdd = 1u << 10;
constexpr int kSignShift = 15;

template <typename T>
__device__ __forceinline__ int clz_t(T x);
template <>
__device__ __forceinline__ int clz_t<uint64_t>(uint64_t x) {
  return __clzll((long long)x);
}
template <>
__device__ __forceinline__ int clz_t<u128>(u128 x) {
  uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
  return hi ? __clzll((long long)hi) : 64 + __clzll((long long)lo);
}

template <typename T>
__device__ __forceinline__ int ctz_t(T x) {
  return __builtin_ctzll((unsigned long long)x);
}

template <typename T>
__device__ __forceinline__ int popc_t(T x) {
  return __popcll((unsigned long long)x);
}

template <typename Code>
__device__ __forceinline__ Code load_code(const Lane& L, int base, int x) {
  if constexpr (sizeof(Code) == 8) {
    return (uint64_t)L.word(base + 2 * x) | ((uint64_t)L.word(base + 2 * x + 1) << 32);
  } else {
    u128 r = 0;
    for (int k = 3; k >= 0; --k) r = (r << 32) | L.word(base + 4 * x + k);
    return r;
  }
}

template <typename Code>
__device__ __forceinline__ void store_code(const Lane& L, int base, int x, Code c) {
  constexpr int W = sizeof(Code) / 4;
  for (int k = 0; k < W; ++k) L.word(base + W * x + k) = (uint32_t)(c >> (32 * k));
}

template <typename Adj>
__device__ __forceinline__ Adj load_adj(const Lane& L, int base, int x) {
  if constexpr (sizeof(Adj) == 4) {
    return L.word(base + x);
  } else {
    return (uint64_t)L.word(base + 2 * x) | ((uint64_t)L.word(base + 2 * x + 1) << 32);
  }
}

template <typename Adj>
__device__ __forceinline__ void store_adj(const Lane& L, int base, int x, Adj a) {
  if constexpr (sizeof(Adj) == 4) {
    L.word(base + x) = a;
  } else {
    L.word(base + 2 * x) = (uint32_t)a;
    L.word(base + 2 * x + 1) = (uint32_t)(a >> 32);
  }
}

// ------------------------------------------------------------- one mask

template <int D>
struct Eval {
  using C = Cfg<D>;
  using Mask = typename C::Mask;
  using Adj = typename C::Adj;
  using Code = typename C::Code;

  __device__ static __forceinline__ uint32_t bit(Mask m, int p) { return (uint32_t)(m >> p) & 1u; }

  // root of u (walk only), starting from its entry eu
  __device__ static __forceinline__ int find(const Lane& L, int u, uint32_t eu, uint32_t& er) {
    int r = (int)(eu & kParent);
    er = eu;
    if (r != u) {
      er = L.ent(r);
      while ((int)(er & kParent) != r) {
        r = (int)(er & kParent);
        er = L.ent(r);
      }
    }
    return r;
  }

  // root and parity of u relative to its root
  __device__ static __forceinline__ int find_parity(const Lane& L, int u, uint32_t& er, uint32_t& par) {
    int r = u;
    er = L.ent(u);
    par = 0;
    while ((int)(er & kParent) != r) {
      par ^= (er & kParity) ? 1u : 0u;
      r = (int)(er & kParent);
      er = L.ent(r);
    }
    return r;
  }

  // Returns the scheme code (0 on a failed consistency check, with the
  // reason or-ed into errs).
  __device__ static u128 run(const uint32_t* __restrict__ prog, Mask m, const Lane& L, uint32_t& errs) {
    const uint32_t* nbr = prog + C::NV;
    const uint32_t* pairs = prog + C::NV + C::NE;

    // ---- phase 1: components of same-sign vertices
    for (int v = 0; v < C::NV; ++v) {
      const uint32_t rec = prog[v];
      const int p = rec & 0x7F;
      const uint32_t sv = bit(m, p) ^ ((rec >> 7) & 1u);
      const int nn = (rec >> 8) & 0xFF;
      const int off = rec >> 16;
      int rv = v;
      for (int k = 0; k < nn; ++k) {
        const int u = (int)nbr[off + k];
        const uint32_t eu = L.ent(u);
        if ((eu >> kSignShift) == sv) {
          uint32_t er;
          const int r = find(L, u, eu, er);
          if (r != (int)(eu & kParent)) L.ent(u) = (uint16_t)((eu & ~kParent) | (uint32_t)r);
          if (rv == v) {
            rv = r;
          } else if (r != rv) {
            const int lo = r < rv ? r : rv, hi = r < rv ? rv : r;
            L.ent(hi) = (uint16_t)((sv << kSignShift) | (uint32_t)lo);
            rv = lo;
          }
        }
      }
      L.ent(v) = (uint16_t)((sv << kSignShift) | (uint32_t)rv);
    }

    // ---- phase 2: regions (antipodal identification)
    for (int t = 0; t < C::NP; ++t) {
      const uint32_t pr = pairs[t];
      const int a = pr & 0xFFFF, b = pr >> 16;
      uint32_t ea, eb, pa, pb;
      const int ra = find_parity(L, a, ea, pa);
      const int rb = find_parity(L, b, eb, pb);
      if (ra == rb) {
        if (C::EVEN && pa == pb) L.ent(ra) = (uint16_t)(ea | kOdd);
      } else {
        const bool a_lo = ra < rb;
        const int lo = a_lo ? ra : rb, hi = a_lo ? rb : ra;
        const uint32_t elo = a_lo ? ea : eb, ehi = a_lo ? eb : ea;
        const uint32_t par = C::EVEN ? ((pa ^ pb ^ 1u) ? kParity : 0u) : 0u;
        L.ent(hi) = (uint16_t)((ehi & (1u << kSignShift)) | par | (uint32_t)lo);
        if (ehi & kOdd) L.ent(lo) = (uint16_t)(elo | kOdd);
      }
    }

    // ---- phase 3: region ids and adjacency
    int nR = 0;
    int root = -1;
    uint32_t err = 0;
    for (int v = 0; v < C::NV; ++v) {
      const uint32_t rec = prog[v];
      const int nn = (rec >> 8) & 0xFF;
      const int off = rec >> 16;
      const uint32_t ev = L.ent(v);
      const uint32_t sv = ev >> kSignShift;
      const int p = (int)(ev & kParent);
      int cid;
      if (p == v) {
        cid = nR < C::RMAX ? nR : C::RMAX - 1;
        err |= nR < C::RMAX ? 0u : kErrRegions;
        ++nR;
        store_adj<Adj>(L, C::ADJ_BASE, cid, (Adj)0);
        if (C::EVEN && (ev & kOdd)) {
          if (root >= 0) err |= kErrRoot;
          root = cid;
        }
      } else {
        cid = (int)(L.ent(p) & kParent);
      }
      Adj nb = 0;
      for (int k = 0; k < nn; ++k) {
        const int u = (int)nbr[off + k];
        const uint32_t eu = L.ent(u);
        if ((eu >> kSignShift) != sv) {
          const int cu = (int)(eu & kParent);
          if (cu == cid) {
            if (C::EVEN) {
              err |= kErrSelfLoop;
            } else {
              if (root >= 0 && root != cid) err |= kErrRoot;
              root = cid;
            }
          } else {
            nb |= (Adj)1 << cu;
          }
        }
      }
      L.ent(v) = (uint16_t)((sv << kSignShift) | (uint32_t)cid);
      if (nb) {
        store_adj<Adj>(L, C::ADJ_BASE, cid, load_adj<Adj>(L, C::ADJ_BASE, cid) | nb);
        Adj t = nb;
        while (t) {
          const int a = ctz_t(t);
          t &= t - 1;
          store_adj<Adj>(L, C::ADJ_BASE, a, load_adj<Adj>(L, C::ADJ_BASE, a) | ((Adj)1 << cid));
        }
      }
    }
    if (root < 0) err |= kErrRoot;
    if (nR > C::RMAX) nR = C::RMAX;
    if (err) {
      errs |= err;
      return 0;
    }

    // ---- phase 4: breadth-first order from the root, then AHU codes
    // tree check: number of adjacency bits = 2 (nR - 1)
    int deg2 = 0;
    for (int x = 0; x < nR; ++x) deg2 += popc_t(load_adj<Adj>(L, C::ADJ_BASE, x));
    if (deg2 != 2 * (nR - 1)) {
      errs |= kErrTree;
      return 0;
    }
    Adj visited = (Adj)1 << root;
    L.byte(C::ORD_BASE + 0, 0) = (uint8_t)root;
    L.byte(C::ORD_BASE + root, 1) = 0xFF;
    int head = 0, tail = 1;
    while (head < tail) {
      const int x = L.byte(C::ORD_BASE + head, 0);
      ++head;
      Adj nb = load_adj<Adj>(L, C::ADJ_BASE, x) & ~visited;
      visited |= nb;
      while (nb) {
        const int y = ctz_t(nb);
        nb &= nb - 1;
        L.byte(C::ORD_BASE + tail, 0) = (uint8_t)y;
        L.byte(C::ORD_BASE + y, 1) = (uint8_t)x;
        ++tail;
      }
    }
    if (tail != nR) {
      errs |= kErrTree;
      return 0;
    }
    Adj leaves = 0;
    Code word = 0;
    int wlen = 0;
    for (int i = nR - 1; i >= 0; --i) {
      const int x = L.byte(C::ORD_BASE + i, 0);
      const int px = L.byte(C::ORD_BASE + x, 1);
      Adj kids = load_adj<Adj>(L, C::ADJ_BASE, x);
      if (i > 0) kids &= ~((Adj)1 << px);
      if (kids == 0) {
        leaves |= (Adj)1 << x;
        continue;
      }
      Adj rest = kids & ~leaves;
      const int nleaf = popc_t(kids & leaves);
      Code acc = 0;
      int len = 0;
      while (rest) {
        int best = -1;
        Code bkey = 0, bcode = 0;
        Adj t = rest;
        while (t) {
          const int y = ctz_t(t);
          t &= t - 1;
          const Code cy = load_code<Code>(L, C::CODE_BASE, y);
          const Code ky = cy << clz_t(cy);
          if (best < 0 || ky > bkey) {
            best = y;
            bkey = ky;
            bcode = cy;
          }
        }
        rest &= ~((Adj)1 << best);
        const int lb = (int)(8 * sizeof(Code)) - clz_t(bcode);
        acc = (acc << lb) | bcode;
        len += lb;
      }
      if (nleaf) {
        const Code pat = (~(Code)0 / 3) << 1;  // ...101010
        acc = (acc << (2 * nleaf)) | (pat >> (8 * (int)sizeof(Code) - 2 * nleaf));
        len += 2 * nleaf;
      }
      if (i > 0) {
        store_code<Code>(L, C::CODE_BASE, x, ((Code)1 << (len + 1)) | (acc << 1));
      } else {
        word = acc;
        wlen = len;
      }
    }
    u128 code = ((u128)1 << wlen) | (u128)word;
    if (!C::EVEN) code |= (u128)1 << 127;
    return code;
  }
};

// ---------------------------------------------------------------- masks

template <int D>
__device__ __forceinline__ typename Cfg<D>::Mask load_mask(const void* __restrict__ masks, int64_t i) {
  constexpr int B = mask_bytes(D);
  if constexpr (B == 4) {
    return (uint64_t)static_cast<const uint32_t*>(masks)[i];
  } else if constexpr (B == 8) {
    return static_cast<const uint64_t*>(masks)[i];
  } else {
    const uint64_t* p = static_cast<const uint64_t*>(masks) + 2 * i;
    return ((u128)p[1] << 64) | (u128)p[0];
  }
}

struct Runs {
  int n;
  uint8_t src[8], len[8], dst[8];
};

// Runs unpacked into wave-uniform scalars once per kernel.
struct RunRegs {
  int n;
  int src[8], dst[8];
  uint64_t keep[8];
};

__device__ __forceinline__ RunRegs unpack_runs(const Runs& r) {
  RunRegs q;
  q.n = r.n;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    q.src[k] = r.src[k];
    q.dst[k] = r.dst[k];
    q.keep[k] = r.len[k] >= 64 ? ~0ull : ((1ull << r.len[k]) - 1);
  }
  return q;
}

template <typename Mask>
__device__ __forceinline__ Mask deposit(uint64_t idx, const RunRegs& r) {
  Mask m = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k < r.n) m |= (Mask)((idx >> r.src[k]) & r.keep[k]) << r.dst[k];
  return m;
}

// ------------------------------------------------------------ histograms

struct HistDev {
  uint32_t* state;  // 0 empty, 1 being filled, 2 ready
  uint64_t* key;    // 2 per slot (lo, hi)
  uint64_t* cnt;
  uint64_t* wit;
  uint32_t* overflow;
  uint32_t cap_mask;
};

__device__ __forceinline__ uint32_t hash_code(uint64_t lo, uint64_t hi) {
  uint64_t z = lo ^ (hi * 0x9E3779B97F4A7C15ull) ^ 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 29)) * 0x94D049BB133111EBull;
  return (uint32_t)(z ^ (z >> 32));
}

// Insert (lo,hi) += k, witness min.  A slot goes 0 -> 1 (claimed by one
// lane's CAS) -> 2 (key, count and witness written, released).  A lane that
// meets a slot in state 1 re-reads it until the claiming lane has
// published it (a handful of stores, so the wait is short); after
// kClaimWait reads it moves on instead, which can only leave a duplicate
// key that pw_hist_read merges.
constexpr int kClaimWait = 1 << 16;

__device__ void global_insert(const HistDev& h, uint64_t lo, uint64_t hi, uint64_t k, uint64_t w) {
  uint32_t s = hash_code(lo, hi) & h.cap_mask;
  int waited = 0;
  for (uint32_t probe = 0; probe <= h.cap_mask;) {
    uint32_t st = __hip_atomic_load(&h.state[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (st == 0) {
      uint32_t expected = 0;
      if (__hip_atomic_compare_exchange_strong(&h.state[s], &expected, 1u, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        h.key[2 * s] = lo;
        h.key[2 * s + 1] = hi;
        h.cnt[s] = k;
        h.wit[s] = w;
        __hip_atomic_store(&h.state[s], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
      st = expected;
    }
    if (st == 1 && ++waited < kClaimWait) continue;  // same slot again
    if (st == 2 && h.key[2 * s] == lo && h.key[2 * s + 1] == hi) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&h.cnt[s]), (unsigned long long)k);
      atomicMin(reinterpret_cast<unsigned long long*>(&h.wit[s]), (unsigned long long)w);
      return;
    }
    waited = 0;
    ++probe;
    s = (s + 1) & h.cap_mask;
  }
  atomicOr(h.overflow, 1u);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Per-wave code table held in registers: two entries per lane, 128 per
// wave.  Every member is called by the whole wave with uniform arguments.
struct Slot {
  uint64_t lo, hi, cnt, wit;  // lo = hi = 0: empty (valid codes are never 0)
  __device__ __forceinline__ bool holds(uint64_t a, uint64_t b) const { return lo == a && hi == b; }
  __device__ __forceinline__ bool empty() const { return (lo | hi) == 0; }
  __device__ __forceinline__ void put(uint64_t a, uint64_t b, uint64_t k, uint64_t w) {
    lo = a;
    hi = b;
    cnt = k;
    wit = w;
  }
  __device__ __forceinline__ void bump(uint64_t k, uint64_t w) {
    cnt += k;
    wit = w < wit ? w : wit;
  }
};

struct WaveTable {
  Slot s0, s1;

  __device__ __forceinline__ void clear() {
    s0.put(0, 0, 0, 0);
    s1.put(0, 0, 0, 0);
  }

  __device__ __forceinline__ void flush(const HistDev& h) {
    if (!s0.empty()) global_insert(h, s0.lo, s0.hi, s0.cnt, s0.wit);
    if (!s1.empty()) global_insert(h, s1.lo, s1.hi, s1.cnt, s1.wit);
    clear();
  }

  __device__ __forceinline__ void add(uint64_t lo, uint64_t hi, uint64_t k, uint64_t w, int lane,
                                      const HistDev& h) {
    const bool h0 = s0.holds(lo, hi), h1 = s1.holds(lo, hi);
    if (__ballot(h0 || h1)) {
      if (h0) s0.bump(k, w);
      if (h1) s1.bump(k, w);
      return;
    }
    const uint64_t e0 = __ballot(s0.empty());
    if (e0) {
      if (lane == __ffsll((unsigned long long)e0) - 1) s0.put(lo, hi, k, w);
      return;
    }
    const uint64_t e1 = __ballot(s1.empty());
    if (e1) {
      if (lane == __ffsll((unsigned long long)e1) - 1) s1.put(lo, hi, k, w);
      return;
    }
    flush(h);
    if (lane == 0) s0.put(lo, hi, k, w);
  }

  // Aggregate one batch (one code per lane, `valid` lanes only).  Lanes
  // hold consecutive indices, so the lowest lane of a match carries the
  // smallest witness.
  __device__ __forceinline__ void add_batch(uint64_t lo, uint64_t hi, bool valid, uint64_t widx, int lane,
                                            const HistDev& h) {
    uint64_t act = __ballot(valid && (lo | hi) != 0);
    while (act) {
      const int L = __ffsll((unsigned long long)act) - 1;
      const uint64_t clo = readlane64(lo, L), chi = readlane64(hi, L);
      const uint64_t match = __ballot(lo == clo && hi == chi) & act;
      const uint64_t w = readlane64(widx, L);
      add(clo, chi, (uint64_t)__popcll((unsigned long long)match), w, lane, h);
      act &= ~match;
    }
  }
};


// ---------------------------------------------------------------- kernels

template <int D>
__global__ __launch_bounds__(256) void k_codes(const uint32_t* __restrict__ prog, const void* __restrict__ masks,
                                               int64_t n, uint64_t* __restrict__ codes,
                                               uint32_t* __restrict__ errflag) {
  using C = Cfg<D>;
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Lane L{smem + wave * C::LANE_WORDS * 64 + lane};
  uint32_t errs = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    const typename C::Mask m = valid ? load_mask<D>(masks, i) : (typename C::Mask)0;
    const u128 code = Eval<D>::run(prog, m, L, errs);
    if (valid) {
      codes[2 * i] = (uint64_t)code;
      codes[2 * i + 1] = (uint64_t)(code >> 64);
    }
  }
  if (errs) atomicOr(errflag, errs);
}

template <int D>
__global__ __launch_bounds__(256) void k_hist(const uint32_t* __restrict__ prog, const void* __restrict__ masks,
                                              int64_t n, uint64_t index_base, HistDev h,
                                              uint32_t* __restrict__ errflag) {
  using C = Cfg<D>;
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Lane L{smem + wave * C::LANE_WORDS * 64 + lane};
  WaveTable tab;
  tab.clear();
  uint32_t errs = 0;
  const int64_t waves_total = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64; base < n; base += waves_total * 64) {
    const int64_t i = base + lane;
    const bool valid = i < n;
    const typename C::Mask m = valid ? load_mask<D>(masks, i) : (typename C::Mask)0;
    const u128 code = Eval<D>::run(prog, m, L, errs);
    tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, index_base + (uint64_t)i, lane, h);
  }
  tab.flush(h);
  if (errs) atomicOr(errflag, errs);
}

template <int D>
__global__ __launch_bounds__(256) void k_enum(const uint32_t* __restrict__ prog, uint64_t first, uint64_t count,
                                              Runs runs, HistDev h, uint32_t* __restrict__ errflag) {
  using C = Cfg<D>;
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Lane L{smem + wave * C::LANE_WORDS * 64 + lane};
  WaveTable tab;
  tab.clear();
  const RunRegs rr = unpack_runs(runs);
  uint32_t errs = 0;
  const uint64_t waves_total = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64; base < count;
       base += waves_total * 64) {
    const uint64_t k = base + lane;
    const bool valid = k < count;
    const uint64_t idx = first + k;
    const typename C::Mask m = deposit<typename C::Mask>(idx, rr);
    const u128 code = Eval<D>::run(prog, m, L, errs);
    tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, idx, lane, h);
  }
  tab.flush(h);
  if (errs) atomicOr(errflag, errs);
}

}  // namespace pw

// =================================================================== host

using namespace pw;

struct pw_tri {
  HostProgram prog;
  uint32_t* d_prog = nullptr;
  uint32_t* d_err = nullptr;
  int device = 0;
};

struct pw_hist {
  int32_t cap = 0;
  uint32_t* state = nullptr;
  uint64_t* key = nullptr;
  uint64_t* cnt = nullptr;
  uint64_t* wit = nullptr;
  uint32_t* overflow = nullptr;
  HistDev dev() const { return HistDev{state, key, cnt, wit, overflow, (uint32_t)(cap - 1)}; }
};

namespace {

thread_local char g_err[512] = "";

__attribute__((format(printf, 2, 3))) pw_status set_err(pw_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define PW_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return set_err(PW_ERR_HIP, "%s (code %d)", hipGetErrorString(e_), (int)e_); \
  } while (0)

int cu_count() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
  }
  return n;
}

// Enough blocks to fill every CU once (the LDS footprint bounds how many
// blocks a CU holds); each wave then loops over many batches.
template <int D>
int blocks_for(int64_t units_per_block, int64_t n) {
  using C = Cfg<D>;
  const int64_t lds = (int64_t)C::LANE_WORDS * 4 * 64 * C::WAVES;
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / lds));
  const int64_t need = (n + units_per_block - 1) / units_per_block;
  return (int)std::max<int64_t>(1, std::min(need, (int64_t)cu_count() * per_cu));
}

template <int D>
pw_status launch_codes(const pw_tri* t, const void* masks, int64_t n, uint64_t* codes, hipStream_t s) {
  using C = Cfg<D>;
  const int threads = 64 * C::WAVES;
  const size_t lds = (size_t)C::LANE_WORDS * 4 * 64 * C::WAVES;
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_codes<D>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  hipLaunchKernelGGL(k_codes<D>, dim3(blocks_for<D>(threads, n)), dim3(threads), lds, s, t->d_prog, masks, n,
                     codes, t->d_err);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template <int D>
pw_status launch_hist(const pw_tri* t, const void* masks, int64_t n, uint64_t base, const pw_hist* h,
                      hipStream_t s) {
  using C = Cfg<D>;
  const int threads = 64 * C::WAVES;
  const size_t lds = (size_t)C::LANE_WORDS * 4 * 64 * C::WAVES;
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hist<D>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  hipLaunchKernelGGL(k_hist<D>, dim3(blocks_for<D>(threads, n)), dim3(threads), lds, s, t->d_prog, masks, n, base,
                     h->dev(), t->d_err);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template <int D>
pw_status launch_enum(const pw_tri* t, uint64_t first, uint64_t count, const Runs& runs, const pw_hist* h,
                      hipStream_t s) {
  using C = Cfg<D>;
  const int threads = 64 * C::WAVES;
  const size_t lds = (size_t)C::LANE_WORDS * 4 * 64 * C::WAVES;
  static std::once_flag once;
  std::call_once(once, [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_enum<D>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  const int64_t n = count > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)count;
  hipLaunchKernelGGL(k_enum<D>, dim3(blocks_for<D>(threads, n)), dim3(threads), lds, s, t->d_prog, first, count,
                     runs, h->dev(), t->d_err);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

#define PW_DISPATCH(d, F, ...)                \
  switch (d) {                                \
    case 1: return F<1>(__VA_ARGS__);         \
    case 2: return F<2>(__VA_ARGS__);         \
    case 3: return F<3>(__VA_ARGS__);         \
    case 4: return F<4>(__VA_ARGS__);         \
    case 5: return F<5>(__VA_ARGS__);         \
    case 6: return F<6>(__VA_ARGS__);         \
    case 7: return F<7>(__VA_ARGS__);         \
    case 8: return F<8>(__VA_ARGS__);         \
    case 9: return F<9>(__VA_ARGS__);         \
    case 10: return F<10>(__VA_ARGS__);       \
    case 11: return F<11>(__VA_ARGS__);       \
    case 12: return F<12>(__VA_ARGS__);       \
    default: return set_err(PW_ERR_ARG, "degree %d out of range", (int)(d)); \
  }

}  // namespace

extern "C" {

const char* pw_last_error(void) { return g_err; }

int32_t pw_version(void) { return 100; }

int32_t pw_mask_bytes(int32_t d) {
  if (d < 1 || d > kDMax) return PW_ERR_ARG;
  return mask_bytes(d);
}

pw_status pw_tri_create(int32_t d, const int16_t* edges_ij, int32_t n_edges, pw_tri_t* out) {
  if (!out) return set_err(PW_ERR_ARG, "null output handle");
  *out = nullptr;
  pw_tri* t = new (std::nothrow) pw_tri();
  if (!t) return set_err(PW_ERR_ARG, "out of host memory");
  char msg[256];
  int rc = build_program(d, edges_ij, n_edges, &t->prog, msg, sizeof msg);
  if (rc != 0) {
    delete t;
    return set_err(rc, "%s", msg);
  }
  hipError_t e = hipGetDevice(&t->device);
  if (e == hipSuccess) e = hipMalloc(&t->d_prog, sizeof(uint32_t) * t->prog.n_words);
  if (e == hipSuccess) e = hipMalloc(&t->d_err, sizeof(uint32_t));
  if (e == hipSuccess)
    e = hipMemcpy(t->d_prog, t->prog.words, sizeof(uint32_t) * t->prog.n_words, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(t->d_err, 0, sizeof(uint32_t));
  if (e != hipSuccess) {
    if (t->d_prog) (void)hipFree(t->d_prog);
    if (t->d_err) (void)hipFree(t->d_err);
    delete t;
    return set_err(PW_ERR_HIP, "%s (code %d)", hipGetErrorString(e), (int)e);
  }
  *out = t;
  return PW_OK;
}

pw_status pw_tri_destroy(pw_tri_t t) {
  if (!t) return PW_OK;
  (void)hipFree(t->d_prog);
  (void)hipFree(t->d_err);
  delete t;
  return PW_OK;
}

pw_status pw_tri_info(pw_tri_t t, int32_t* d, int32_t* n_points_, int32_t* n_vertices_, int32_t* n_diamond_edges_,
                      int32_t* n_pairs) {
  if (!t) return set_err(PW_ERR_ARG, "null handle");
  if (d) *d = t->prog.d;
  if (n_points_) *n_points_ = t->prog.nA;
  if (n_vertices_) *n_vertices_ = t->prog.nV;
  if (n_diamond_edges_) *n_diamond_edges_ = t->prog.nE;
  if (n_pairs) *n_pairs = t->prog.nP;
  return PW_OK;
}

pw_status pw_tri_errors(pw_tri_t t, uint32_t* flags) {
  if (!t || !flags) return set_err(PW_ERR_ARG, "null argument");
  PW_HIP(hipDeviceSynchronize());
  PW_HIP(hipMemcpy(flags, t->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost));
  PW_HIP(hipMemset(t->d_err, 0, sizeof(uint32_t)));
  return PW_OK;
}

pw_status patchwork_scheme_batch(pw_tri_t t, const void* masks, int64_t n, uint64_t* codes, hipStream_t s) {
  if (!t) return set_err(PW_ERR_ARG, "null handle");
  if (n < 0) return set_err(PW_ERR_ARG, "negative mask count %lld", (long long)n);
  if (n == 0) return PW_OK;
  if (!masks || !codes) return set_err(PW_ERR_ARG, "null device buffer");
  PW_DISPATCH(t->prog.d, launch_codes, t, masks, n, codes, s);
}

pw_status pw_hist_create(int32_t capacity, pw_hist_t* out) {
  if (!out) return set_err(PW_ERR_ARG, "null output handle");
  *out = nullptr;
  if (capacity < 16 || capacity > (1 << 26) || (capacity & (capacity - 1)))
    return set_err(PW_ERR_ARG, "histogram capacity must be a power of two in [16, 2^26], got %d", (int)capacity);
  pw_hist* h = new (std::nothrow) pw_hist();
  if (!h) return set_err(PW_ERR_ARG, "out of host memory");
  h->cap = capacity;
  hipError_t e = hipMalloc(&h->state, sizeof(uint32_t) * capacity);
  if (e == hipSuccess) e = hipMalloc(&h->key, sizeof(uint64_t) * 2 * capacity);
  if (e == hipSuccess) e = hipMalloc(&h->cnt, sizeof(uint64_t) * capacity);
  if (e == hipSuccess) e = hipMalloc(&h->wit, sizeof(uint64_t) * capacity);
  if (e == hipSuccess) e = hipMalloc(&h->overflow, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(h->state, 0, sizeof(uint32_t) * capacity);
  if (e == hipSuccess) e = hipMemset(h->overflow, 0, sizeof(uint32_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(h->state);
    (void)hipFree(h->key);
    (void)hipFree(h->cnt);
    (void)hipFree(h->wit);
    (void)hipFree(h->overflow);
    delete h;
    return set_err(PW_ERR_HIP, "%s (code %d)", hipGetErrorString(e), (int)e);
  }
  *out = h;
  return PW_OK;
}

pw_status pw_hist_reset(pw_hist_t h, hipStream_t s) {
  if (!h) return set_err(PW_ERR_ARG, "null handle");
  PW_HIP(hipMemsetAsync(h->state, 0, sizeof(uint32_t) * h->cap, s));
  PW_HIP(hipMemsetAsync(h->overflow, 0, sizeof(uint32_t), s));
  return PW_OK;
}

pw_status pw_hist_destroy(pw_hist_t h) {
  if (!h) return PW_OK;
  (void)hipFree(h->state);
  (void)hipFree(h->key);
  (void)hipFree(h->cnt);
  (void)hipFree(h->wit);
  (void)hipFree(h->overflow);
  delete h;
  return PW_OK;
}

pw_status pw_hist_read(pw_hist_t h, uint64_t* codes, uint64_t* counts, uint64_t* witness, int32_t capacity,
                       int32_t* n_used) {
  if (!h || !n_used) return set_err(PW_ERR_ARG, "null argument");
  if (capacity < 0 || (capacity > 0 && (!codes || !counts || !witness)))
    return set_err(PW_ERR_ARG, "bad output arrays");
  PW_HIP(hipDeviceSynchronize());
  std::vector<uint32_t> st(h->cap);
  std::vector<uint64_t> key(2 * (size_t)h->cap), cnt(h->cap), wit(h->cap);
  uint32_t ovf = 0;
  PW_HIP(hipMemcpy(st.data(), h->state, sizeof(uint32_t) * h->cap, hipMemcpyDeviceToHost));
  PW_HIP(hipMemcpy(key.data(), h->key, sizeof(uint64_t) * 2 * h->cap, hipMemcpyDeviceToHost));
  PW_HIP(hipMemcpy(cnt.data(), h->cnt, sizeof(uint64_t) * h->cap, hipMemcpyDeviceToHost));
  PW_HIP(hipMemcpy(wit.data(), h->wit, sizeof(uint64_t) * h->cap, hipMemcpyDeviceToHost));
  PW_HIP(hipMemcpy(&ovf, h->overflow, sizeof(uint32_t), hipMemcpyDeviceToHost));
  struct Ent {
    uint64_t hi, lo, cnt, wit;
  };
  std::vector<Ent> ents;
  for (int s = 0; s < h->cap; ++s)
    if (st[s] == 2) ents.push_back({key[2 * s + 1], key[2 * s], cnt[s], wit[s]});
  std::sort(ents.begin(), ents.end(),
            [](const Ent& a, const Ent& b) { return a.hi != b.hi ? a.hi < b.hi : a.lo < b.lo; });
  std::vector<Ent> merged;
  for (const Ent& e : ents) {
    if (!merged.empty() && merged.back().hi == e.hi && merged.back().lo == e.lo) {
      merged.back().cnt += e.cnt;
      merged.back().wit = std::min(merged.back().wit, e.wit);
    } else {
      merged.push_back(e);
    }
  }
  *n_used = (int32_t)merged.size();
  const int n = std::min<int>(capacity, (int)merged.size());
  for (int k = 0; k < n; ++k) {
    codes[2 * k] = merged[k].lo;
    codes[2 * k + 1] = merged[k].hi;
    counts[k] = merged[k].cnt;
    witness[k] = merged[k].wit;
  }
  if (ovf) return set_err(PW_ERR_HIST_FULL, "histogram ran out of slots");
  return PW_OK;
}

pw_status patchwork_scheme_histogram(pw_tri_t t, const void* masks, int64_t n, uint64_t index_base, pw_hist_t h,
                                     hipStream_t s) {
  if (!t || !h) return set_err(PW_ERR_ARG, "null handle");
  if (n < 0) return set_err(PW_ERR_ARG, "negative mask count %lld", (long long)n);
  if (n == 0) return PW_OK;
  if (!masks) return set_err(PW_ERR_ARG, "null device buffer");
  PW_DISPATCH(t->prog.d, launch_hist, t, masks, n, index_base, h, s);
}

pw_status patchwork_scheme_enumerate_range(pw_tri_t t, uint64_t first, uint64_t count,
                                           const uint64_t fixed_zero_bits[2], pw_hist_t h, hipStream_t s) {
  if (!t || !h || !fixed_zero_bits) return set_err(PW_ERR_ARG, "null argument");
  const int nA = t->prog.nA;
  Runs runs{};
  int nfree = 0;
  for (int b = 0; b < nA;) {
    const bool fixed = (fixed_zero_bits[b / 64] >> (b % 64)) & 1;
    if (fixed) {
      ++b;
      continue;
    }
    int e = b;
    while (e < nA && !((fixed_zero_bits[e / 64] >> (e % 64)) & 1)) ++e;
    if (runs.n == 8) return set_err(PW_ERR_ARG, "the free bits form more than 8 runs");
    runs.src[runs.n] = (uint8_t)nfree;
    runs.len[runs.n] = (uint8_t)(e - b);
    runs.dst[runs.n] = (uint8_t)b;
    ++runs.n;
    nfree += e - b;
    b = e;
  }
  // only the low 64 index bits are addressable
  for (int k = 0; k < runs.n; ++k) {
    if (runs.src[k] >= 64) {
      runs.n = k;
      break;
    }
    if (runs.src[k] + runs.len[k] > 64) runs.len[k] = (uint8_t)(64 - runs.src[k]);
  }
  if (count == 0) return PW_OK;
  if (nfree < 64) {
    const uint64_t lim = 1ull << nfree;
    if (first >= lim || count > lim - first)
      return set_err(PW_ERR_RANGE, "range exceeds 2^(free bits) (free bits %d)", nfree);
  } else if (first + count < first) {
    return set_err(PW_ERR_RANGE, "range wraps around 2^64");
  }
  PW_DISPATCH(t->prog.d, launch_enum, t, first, count, runs, h, s);
}

}  // extern "C"
