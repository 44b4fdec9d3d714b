// pw_device.h -- device-side building blocks shared by the scheme kernels:
// per-degree configuration, per-lane LDS views, the evaluation of one sign
// mask (Alg. 1 of "Fast Isotopy Computation for T-Curves", Sec. 2), the
// in-kernel mask generator and the two-level code histogram.
//
// LDS layout: each wave owns LANE_WORDS * 64 dwords.  Word k of lane l sits
// at dword k * 64 + l (every lane in its own bank whatever the index); the
// vertex entries of lane l form one contiguous row of E_WORDS (odd) dwords
// starting at dword l * E_WORDS (its own bank for a uniform vertex).  The
// parent table of phases 3-4 is one byte row per region.
//
// Per mask (thread) the phases are:
//   1 components (Alg. 1, its first union-find over the reflected
//     diamond: same-sign vertices joined by uncrossed edges): vertices in
//     program order; each earlier neighbour with the same sign is unioned.
//     Entry of v: the index of its union-find parent (u8 where 7 bits
//     index every vertex: odd d <= 7, even d <= 6; u16 otherwise), for
//     even d with the parity to the parent and, at a root, the odd-cycle
//     flag.  Signs are bits of the mask and are not stored.
//     Links always go from the larger root to the smaller one, so every
//     parent index is smaller than its child's.
//   2 regions (Alg. 1, the components merged across the identified
//     antipodal boundary points): union along the 2d pairs.  For even d the union
//     carries parity 1 (each identification reverses orientation, proof of
//     Thm. 2) and a same-parity closure marks an odd cycle.
//   3 region ids and the region tree: vertices in order again; a root gets
//     the next region id, any other vertex copies the id of its parent
//     (already relabelled because parents are smaller).  The region tree is
//     read off a fixed spanning tree of T<> (each vertex's first earlier
//     neighbour): the first vertex of a region hangs below the region of its
//     tree parent (Alg. 1's region adjacency graph from the crossed edges,
//     restricted to spanning-tree edges, which cross every curve
//     component).  For odd d a crossed tree edge inside one region marks
//     the root (the pseudo-line's region).
//   4 re-root the tree at the root region (Alg. 1 root rule), breadth-first
//     order, canonical code (Alg. 1 last step, AHU encoding): children codes
//     sorted descending by their left-aligned bit strings; leaves ('10')
//     sort last.
#pragma once
#if defined(__HIPCC_RTC__)
// compiled at run time for one triangulation: no standard headers there
typedef __hip_internal::uint8_t uint8_t;
typedef __hip_internal::uint16_t uint16_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::uint64_t uint64_t;
typedef __hip_internal::int64_t int64_t;
#else
#include <hip/hip_runtime.h>

#include <cstdint>
#endif

#include "pw_internal.h"

// an empty asm statement the optimiser cannot see through: pins a value to
// a VGPR at that point of the program (a CPU build of this header may
// define it away)
#ifndef PW_OPAQUE
#define PW_OPAQUE(x) asm volatile("" : "+v"(x))
#endif
// a compiler-only memory barrier: loads and stores are not moved across it
#ifndef PW_FENCE
#define PW_FENCE() asm volatile("" ::: "memory")
#endif
// the same for a wave-uniform value (kept in a scalar register)
#ifndef PW_OPAQUE_S
#define PW_OPAQUE_S(x) asm volatile("" : "+s"(x))
#endif

namespace pw {

typedef unsigned __int128 u128;

// A triangulation's program as the kernels read it.  The batched kernels
// take its address from a descriptor in memory, so the compiler cannot
// tell its address space and would read it with vector loads; in the
// constant address space (read-only during a kernel) its wave-uniform
// words are read through the scalar cache.
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) uint32_t* prog_ptr;
#else
typedef const uint32_t* prog_ptr;
#endif
__device__ __forceinline__ prog_ptr const_prog(const uint32_t* p) { return (prog_ptr)p; }

template <bool B, class X, class Y>
struct cond {
  using type = X;
};
template <class X, class Y>
struct cond<false, X, Y> {
  using type = Y;
};

// ------------------------------------------------------------------ config

// RCAP > 0: the phase-4 tables are sized for at most RCAP regions (a mask
// with more is reported as kErrOverflow and must be evaluated again with
// the full tables); RCAP = 0: sized for the Harnack bound.
template <int D, int RCAP = 0>
struct Cfg {
  static constexpr int NA = n_points(D);
  static constexpr int NV = n_vertices(D);
  static constexpr int NE = n_diamond_edges(D);
  static constexpr int NP = 2 * D;
  static constexpr int RFULL = harnack(D) + 1;  // regions = ovals + 1 <= M + 1
  static constexpr bool CAPPED = RCAP > 0 && RCAP < RFULL;
  static constexpr int RMAX = CAPPED ? RCAP : RFULL;
  static constexpr bool EVEN = (D % 2) == 0;
  using Mask = typename cond<(NA <= 64), uint64_t, u128>::type;
  using Adj = typename cond<(RMAX <= 32), uint32_t, uint64_t>::type;
  // codes of at most RMAX - 1 nodes below the root: 2 (RMAX - 1) bits
  using Code = typename cond<(2 * (RMAX - 1) + 2 <= 64), uint64_t, u128>::type;
  static constexpr int ADJ_W = sizeof(Adj) / 4;
  // vertex entries: u8 where 8 bits index every vertex and the spare
  // entry (d <= 10: BYTE), u16 otherwise (parent index in bits 0-8, for
  // even d the parity to the parent in bit 9 and the odd-cycle flag in
  // bit 10).  Odd d keeps nothing but the index.  Even d with 7-bit
  // indices (d <= 6: NARROW) keeps in bit 7 the parity to the parent at a
  // non-root and the odd-cycle flag at a root (a root has no parent, so
  // the bit is free); even d = 8, 10 (SIDE) keeps that bit in a side
  // bitset of the lane instead (bit v of word SIDE_BASE + v / 32).
  static constexpr bool BYTE = NV + 1 <= 256;
  static constexpr bool NARROW = NV + 1 <= 128;
  static constexpr bool SIDE = EVEN && BYTE && !NARROW;
  using Ent = typename cond<BYTE, uint8_t, uint16_t>::type;
  static constexpr int EB = BYTE ? 1 : 2;
  // a stored region code has 2 * (subtree size) <= 2 * (RMAX - 1) bits
  static constexpr int CODE_W = 2 * (RMAX - 1) <= 32 ? 1 : (int)(sizeof(Code) / 4);
  // per-lane LDS words:
  //   [0, E_WORDS)            vertex entries (phases 1-3) and a spare entry
  //                           (index NV); an odd number of words, so that
  //                           the lanes' entry rows start in distinct banks
  //   [PAR_BASE, +PAR_WORDS)  parent region of every region, one byte row
  //                           of the wave per region (phases 3-4)
  // after phase 3 the entry words hold one slot of SLOT_W words per
  // region: its child mask (ADJ_W words), replaced by its code (CODE_W
  // words) once phase 4 has coded the region -- the mask is read only
  // just before that, and a region's slot is read as a code only by its
  // parent, which is coded later.
  static constexpr int E_WORDS = (((NV + 1) * EB + 3) / 4) | 1;
  static constexpr int SIDE_BASE = E_WORDS;
  static constexpr int SIDE_WORDS = SIDE ? (NV + 1 + 31) / 32 : 0;
  static constexpr int SLOT_W = ADJ_W > CODE_W ? ADJ_W : CODE_W;
  static constexpr int TAIL_WORDS = RMAX * SLOT_W;
  static constexpr int LOW_WORDS = E_WORDS + SIDE_WORDS > TAIL_WORDS ? E_WORDS + SIDE_WORDS : TAIL_WORDS;
  static constexpr int PAR_BASE = LOW_WORDS;
  static constexpr int PAR_WORDS = (RMAX + 4) / 4;  // RMAX byte rows + a spare row
  static constexpr int LANE_WORDS = LOW_WORDS + PAR_WORDS;
  // kernels for one triangulation keep the parent table in a __shared__
  // array of its own (PAR_ROWS byte rows per wave) and the rest in the
  // dynamic area (DYN_WORDS per lane)
  static constexpr int PAR_ROWS = RMAX + 1;
  static constexpr int DYN_WORDS = LOW_WORDS;
  // snapshot area of the sweep kernel: the entries of vertices 0 .. NV-1
  // (SNAP_WORDS words, copied word by word); for even d then the chunk's
  // bitset of the sets that varying vertices reach (TOUCH_WORDS words)
  // and the antipodal pairs left to each batch (2 words), for odd d the
  // words below; padded to 16 bytes
  static constexpr int SNAP_WORDS = (NV * EB + 3) / 4;
  static constexpr int TOUCH_WORDS = EVEN ? (NV + 31) / 32 : 0;
  static constexpr int SNAP_TOUCH = SNAP_WORDS;
  static constexpr int SNAP_KIND = SNAP_TOUCH + TOUCH_WORDS;
  // for odd d instead: the snapshot-root pair of each crossed tree edge
  // between fixed-sign vertices (u16 keys, at most NV edges) and the bitset
  // of the edges whose pair no earlier edge has (HIT_WORDS words)
  static constexpr int HIT_WORDS = EVEN ? 0 : (NV + 31) / 32;
  static constexpr int SNAP_HKEY = SNAP_WORDS;
  static constexpr int SNAP_HX = SNAP_HKEY + (EVEN ? 0 : (2 * NV + 3) / 4);
  static constexpr int SNAP_BYTES = ((EVEN ? SNAP_KIND + 2 : SNAP_HX + HIT_WORDS) * 4 + 15) / 16 * 16;
  static constexpr int WAVE_BYTES = LANE_WORDS * 4 * 64;
  // waves per block: as many waves per CU as the 160 KiB of LDS allows,
  // in blocks of 4 waves, or of 2 where that keeps more of them resident
  // (blocks of one wave measured slower: d = 6, 23 instead of 22 resident
  // waves, 15% slower)
  static constexpr int WAVES_PER_CU = (160 * 1024) / WAVE_BYTES;
  static constexpr int WAVES = WAVES_PER_CU >= 16 ? ((WAVES_PER_CU / 2) * 2 > (WAVES_PER_CU / 4) * 4 ? 2 : 4)
                                                  : (WAVES_PER_CU >= 4 ? 2 : 1);
  // resident waves per SIMD when the LDS is full: the register budget the
  // kernels are compiled for (more registers would lower the occupancy
  // below what the LDS allows)
  static constexpr int RESIDENT = (WAVES_PER_CU / WAVES) * WAVES;
  static constexpr int WAVES_PER_EU = RESIDENT >= 32 ? 8 : (RESIDENT >= 4 ? (RESIDENT + 3) / 4 : 1);
};

// ------------------------------------------------------------ lane memory

// Vertex entries of a lane form one row: entry v at byte lane * 4 * E_WORDS
// + EB * v of the wave's area (EB = 1 or 2 bytes per entry).  An entry
// holds the index of the vertex's union-find parent (phases 1-2; for even d
// also the parity to the parent and, at a root, the odd-cycle flag), then
// its region id (phase 3).  Signs are not stored: the sign of a vertex is a
// fixed bit of the mask.  E_WORDS is odd, so for a uniform v the 64 lanes
// touch 64 distinct banks; divergent parent pointers may share a few.  A
// row is contiguous, so it can be copied a word at a time (the sweep
// kernel's restore).  Word k of a lane (region data, reused entry space)
// sits at byte k * 256 + 4 * lane, and byte row x (the parent table) at
// byte x * 64 + lane.  Entry bytes of one lane overlap words of others:
// phase 4 writes words only after every lane of the wave has finished
// phase 3, which the wave's lockstep execution and program order
// guarantee.
struct Lane {
  uint32_t* w;  // word 0 of this lane; word k at w[k * 64]
  char* e;      // entry 0 of this lane
  char* b;      // byte 0 of this lane in byte rows: byte row x at b[x * 64]
  __device__ __forceinline__ uint32_t& word(int k) const { return w[k * 64]; }
  // word k of the lane's entry row (entries 4 k / EB .. 4 (k + 1) / EB - 1)
  __device__ __forceinline__ uint32_t& eword(int k) const { return reinterpret_cast<uint32_t*>(e)[k]; }
  // byte row x of the parent table
  __device__ __forceinline__ uint8_t& prow(int x) const { return *reinterpret_cast<uint8_t*>(b + x * 64); }
};


template <typename T>
__device__ __forceinline__ int clz_t(T x);
template <>
__device__ __forceinline__ int clz_t<uint32_t>(uint32_t x) {
  return __clz((int)x);
}
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

// ------------------------------------------------------------- one mask

template <int D, int RCAP = 0>
struct Eval {
  using C = Cfg<D, RCAP>;
  using Mask = typename C::Mask;
  using Adj = typename C::Adj;
  using Code = typename C::Code;
  using Ent = typename C::Ent;
  static constexpr uint32_t kIdx = C::NARROW ? 0x7Fu : (C::BYTE ? 0xFFu : 0x1FFu);  // index field of an entry
  // even d: parity to the parent (non-root) and odd-cycle flag (root); one
  // bit in u8 entries, whose meaning the root test decides
  static constexpr uint32_t kParity = C::NARROW ? 0x80u : 0x200u;
  static constexpr uint32_t kOdd = C::NARROW ? 0x80u : 0x400u;
  __device__ static __forceinline__ Adj one(int x) { return (Adj)1 << x; }

  // parent index in an entry (u8 entries of odd d hold nothing else)
  __device__ static __forceinline__ uint32_t idx(uint32_t e) {
    return (C::BYTE && !(C::EVEN && C::NARROW)) ? e : (e & kIdx);
  }

  // ---- the side bitset (SIDE): parity to the parent at a non-root,
  // odd-cycle flag at a root
  __device__ static __forceinline__ uint32_t side_bit(const Lane& L, uint32_t v) {
    return (L.word(C::SIDE_BASE + (int)(v >> 5)) >> (v & 31u)) & 1u;
  }
  __device__ static __forceinline__ void set_side(const Lane& L, uint32_t v, uint32_t b) {
    uint32_t& w = L.word(C::SIDE_BASE + (int)(v >> 5));
    w = (w & ~(1u << (v & 31u))) | (b << (v & 31u));
  }
  // start of an evaluation: no parity or odd-cycle bit set
  __device__ static __forceinline__ void clear_side(const Lane& L) {
    if constexpr (C::SIDE)
      for (int k = 0; k < C::SIDE_WORDS; ++k) L.word(C::SIDE_BASE + k) = 0;
  }
  // odd-cycle flag of root r whose entry is er
  __device__ static __forceinline__ bool odd_flag(const Lane& L, uint32_t r, uint32_t er) {
    if constexpr (C::SIDE) {
      return side_bit(L, r) != 0;
    } else {
      return (er & kOdd) != 0;
    }
  }

  __device__ static __forceinline__ uint32_t bit(Mask m, int p) { return (uint32_t)(m >> p) & 1u; }

  // ---- entries
  __device__ static __forceinline__ Ent& ent(const Lane& L, int v) {
    return *reinterpret_cast<Ent*>(L.e + v * C::EB);
  }
  // end of phase 1 for v: its root so far
  __device__ static __forceinline__ void close(const Lane& L, int v, uint32_t rv) { ent(L, v) = (Ent)rv; }

  // ---- region data (phases 3-4), through a view of the region tables:
  // Lane (one mask per lane) or the view of a lane group (pw_group.h)
  template <class LV>
  __device__ static __forceinline__ int par(const LV& L, int x) {
    return L.prow(x);
  }
  template <class LV>
  __device__ static __forceinline__ void set_par(const LV& L, int x, int p) {
    L.prow(x) = (uint8_t)p;
  }
  template <class LV>
  __device__ static __forceinline__ Adj load_adj(const LV& L, int x) {
    if constexpr (C::ADJ_W == 1) {
      return L.word(C::SLOT_W * x);
    } else {
      return (uint64_t)L.word(C::SLOT_W * x) | ((uint64_t)L.word(C::SLOT_W * x + 1) << 32);
    }
  }
  template <class LV>
  __device__ static __forceinline__ void store_adj(const LV& L, int x, Adj a) {
    if constexpr (C::ADJ_W == 1) {
      L.word(C::SLOT_W * x) = a;
    } else {
      L.word(C::SLOT_W * x) = (uint32_t)a;
      L.word(C::SLOT_W * x + 1) = (uint32_t)(a >> 32);
    }
  }
  template <class LV>
  __device__ static __forceinline__ Code load_code(const LV& L, int x) {
    constexpr int W = C::CODE_W;
    Code r = 0;
    for (int k = W - 1; k >= 0; --k) r = (Code)(r << 32) | (Code)L.word(C::SLOT_W * x + k);
    return r;
  }
  template <class LV>
  __device__ static __forceinline__ void store_code(const LV& L, int x, Code c) {
    constexpr int W = C::CODE_W;
    for (int k = 0; k < W; ++k) L.word(C::SLOT_W * x + k) = (uint32_t)(c >> (32 * k));
  }

  // root of u and u's parity relative to it (parity: even d only)
  __device__ static __forceinline__ uint32_t find_parity(const Lane& L, int u, uint32_t& er, uint32_t& par) {
    uint32_t r = (uint32_t)u;
    er = ent(L, u);
    par = 0;
    while (idx(er) != r) {
      if constexpr (C::SIDE) {
        par ^= side_bit(L, r);
      } else if constexpr (C::EVEN) {
        par ^= (er & kParity) ? 1u : 0u;
      }
      r = idx(er);
      er = ent(L, (int)r);
    }
    return r;
  }

  // Phase 1 step: v's earlier neighbour u; sv, su = signs of v and u, rv =
  // v's root so far (v itself until v is linked).  During phase 1 an entry
  // is a bare parent index.  Written without branches apart from the walk
  // to the root: every lane finds u's root (and points u straight at it),
  // and a lane whose signs differ stores into v's own entry instead -- that
  // entry is scratch until close() writes it, and no walk reaches v before
  // that (every root found is an earlier vertex).
  __device__ static __forceinline__ void edge(const Lane& L, uint32_t sv, uint32_t su, int v, uint32_t& rv, int u) {
    uint32_t r = ent(L, u);
    uint32_t er = ent(L, (int)r);
    while (er != r) {
      r = er;
      er = ent(L, (int)r);
    }
    ent(L, u) = (Ent)r;
    const bool same = su == sv;
    const uint32_t lo = r < rv ? r : rv, hi = r < rv ? rv : r;
    // same sign: the larger root hangs below the smaller one (a no-op
    // rewrite when r == rv; v's own entry when v is still its own root)
    int w = same ? (int)hi : v;
    PW_OPAQUE(w);  // select the index, then address it (one shift-add)
    ent(L, w) = (Ent)lo;
    rv = same ? lo : rv;
  }

  // Phase 1 step of the specialised kernels: as edge(), but the walk starts
  // from ru, a register holding a root u had at some earlier time (u's root
  // when u was closed, refreshed by each later walk from u), so the first
  // LDS read does not wait for another one.  ru is refreshed with u's
  // current root; nothing is written back to u's entry.
  __device__ static __forceinline__ void edge_r(const Lane& L, uint32_t sv, uint32_t su, int v, uint32_t& rv,
                                                uint32_t& ru) {
    uint32_t r = ru;
    uint32_t er = ent(L, (int)r);
    while (er != r) {
      r = er;
      er = ent(L, (int)r);
    }
    ru = r;
    const bool same = su == sv;
    const uint32_t lo = r < rv ? r : rv, hi = r < rv ? rv : r;
    int w = same ? (int)hi : v;
    PW_OPAQUE(w);
    ent(L, w) = (Ent)lo;
    rv = same ? lo : rv;
  }

  // Phase 1 step for a vertex v processed out of index order (the sweep
  // kernel that restores a shared snapshot first): v's entry already holds
  // v, so v may become the smaller root of a union; a lane whose signs
  // differ stores into the spare entry row NV instead.  rv = v's root so far,
  // ru = a root u had at some earlier time (refreshed).
  __device__ static __forceinline__ void edge_v(const Lane& L, uint32_t sv, uint32_t su, int v, uint32_t& rv,
                                                uint32_t& ru) {
    uint32_t r = ru;
    uint32_t er = ent(L, (int)r);
    while (er != r) {
      r = er;
      // (a plain 32-bit index: narrowed to 8 bits, every step would mask)
      PW_OPAQUE(r);
      er = ent(L, (int)r);
    }
    const bool same = su == sv;
    const uint32_t lo = r < rv ? r : rv, hi = r < rv ? rv : r;
    int w = same ? (int)hi : C::NV;
    PW_OPAQUE(w);
    ent(L, w) = (Ent)lo;
    rv = same ? lo : rv;
    ru = same ? lo : r;
  }

  // root of the vertex whose walk starts at r (phase 1 entries)
  __device__ static __forceinline__ uint32_t root(const Lane& L, uint32_t r) {
    uint32_t er = ent(L, (int)r);
    while (er != r) {
      r = er;
      er = ent(L, (int)r);
    }
    return r;
  }

  // Phase 2 step: one antipodal pair (a, b).
  __device__ static __forceinline__ void pair(const Lane& L, int a, int b) {
    uint32_t ea, eb, pa, pb;
    const uint32_t ra = find_parity(L, a, ea, pa);
    const uint32_t rb = find_parity(L, b, eb, pb);
    join(L, ra, rb, ea, eb, pa, pb);
  }

  // The same, telling what the pair did: 1 if it joined two sets, 2 if it
  // set the odd-cycle flag of a set that had none (even d), 0 if it
  // changed nothing.  (The sweep kernel's per-chunk reduction of the pairs
  // whose vertices are all of fixed sign.)
  __device__ static __forceinline__ uint32_t pair_kind(const Lane& L, int a, int b) {
    uint32_t ea, eb, pa, pb;
    const uint32_t ra = find_parity(L, a, ea, pa);
    const uint32_t rb = find_parity(L, b, eb, pb);
    const uint32_t kind = ra != rb ? 1u : ((C::EVEN && pa == pb && !odd_flag(L, ra, ea)) ? 2u : 0u);
    join(L, ra, rb, ea, eb, pa, pb);
    return kind;
  }

  // root of the set of r (an entry's parity and flag bits ignored)
  __device__ static __forceinline__ uint32_t root_of(const Lane& L, uint32_t r) {
    uint32_t er = ent(L, (int)r);
    while (idx(er) != r) {
      r = idx(er);
      er = ent(L, (int)r);
    }
    return r;
  }

  // sets the odd-cycle flag of the set of u (even d): what a pair inside
  // one set closing an odd cycle does
  __device__ static __forceinline__ void odd_mark(const Lane& L, int u) {
    const uint32_t r = root_of(L, (uint32_t)u);
    if constexpr (C::SIDE) {
      set_side(L, r, 1u);
    } else {
      ent(L, (int)r) = (Ent)(ent(L, (int)r) | kOdd);
    }
  }

  // the pair's effect once the roots ra, rb of its vertices and their
  // parities pa, pb (even d) are known: an odd cycle flags the root, else
  // the larger root is linked below the smaller one with the parity that
  // makes the two vertices opposite, passing on its odd-cycle flag
  __device__ static __forceinline__ void join(const Lane& L, uint32_t ra, uint32_t rb, uint32_t ea, uint32_t eb,
                                              uint32_t pa, uint32_t pb) {
    if constexpr (C::SIDE) {
      if (ra == rb) {
        if (pa == pb) set_side(L, ra, 1u);
      } else {
        const uint32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        const uint32_t odd_hi = side_bit(L, hi);  // hi's bit: its odd-cycle flag, then its parity
        ent(L, (int)hi) = (Ent)lo;
        set_side(L, hi, pa ^ pb ^ 1u);
        if (odd_hi) set_side(L, lo, 1u);
      }
    } else if (ra == rb) {
      if (C::EVEN && pa == pb) ent(L, (int)ra) = (Ent)(ea | kOdd);
    } else {
      const bool a_lo = ra < rb;
      const uint32_t lo = a_lo ? ra : rb, hi = a_lo ? rb : ra;
      const uint32_t elo = a_lo ? ea : eb, ehi = a_lo ? eb : ea;
      const uint32_t par = C::EVEN ? ((pa ^ pb ^ 1u) ? kParity : 0u) : 0u;
      ent(L, (int)hi) = (Ent)(par | lo);
      if (C::EVEN && (ehi & kOdd)) ent(L, (int)lo) = (Ent)(elo | kOdd);
    }
  }

  // Phase 3 step for vertex v with spanning-tree parent t (t < 0 for v = 0);
  // sv, st = signs of v and t.  A union-find root is the first vertex of its
  // region and gets the next id.  The tree edges t(v)-v form a spanning
  // tree of T<>.  Each oval separates two regions that both contain
  // vertices, so some tree edge crosses it; the tree edge into the first
  // vertex of a region B comes from the region across one of B's boundary
  // ovals, and "parent(B) = region of t(first vertex of B)" is exactly the
  // region adjacency tree, rooted at the region of vertex 0.  The root of
  // Alg. 1 is collected in `roots` as a set of region ids: for odd d the
  // regions containing a crossed tree edge (an edge crossing the
  // pseudo-line inside one region), for even d the regions whose union-find
  // root carries the odd-cycle flag; finish() requires exactly one.  The
  // entry of v becomes its region id.  Branch-free: a vertex that is not a
  // root stores its (unused) parent-region byte into the spare row RMAX of
  // the parent table.
  __device__ static __forceinline__ void vertex3(const Lane& L, int v, int t, uint32_t sv, uint32_t st, int& nR,
                                                 Adj& roots) {
    vertex3e(L, v, t, sv, st, ent(L, v), nR, roots);
  }

  // the same with v's entry ev read in advance (phase 3 rewrites only the
  // entries of vertices already done, so it may be read any time after
  // phase 2)
  __device__ static __forceinline__ void vertex3e(const Lane& L, int v, int t, uint32_t sv, uint32_t st,
                                                  uint32_t ev, int& nR, Adj& roots) {
    const uint32_t p = idx(ev);
    const bool is_root = p == (uint32_t)v;
    const uint32_t ep = ent(L, (int)p);  // p < v holds its region id already; a root reads its own entry
    const uint32_t et = ent(L, t < 0 ? 0 : t);
    // ids past the Harnack bound share the spare slot RMAX; finish()
    // rejects such a mask (nR > RMAX) before reading any region data
    const int cid = is_root ? (nR < C::RMAX ? nR : C::RMAX) : (int)ep;
    nR += is_root ? 1 : 0;
    // keep the running count a plain running count (re-associating the
    // chain of increments would hold every vertex's flag in a register)
    PW_OPAQUE(nR);
    const bool hit = C::EVEN ? (is_root && odd_flag(L, (uint32_t)v, ev)) : (t >= 0 && st != sv && (int)et == cid);
    roots |= hit ? one(cid & (8 * (int)sizeof(Adj) - 1)) : (Adj)0;
    const uint32_t pc = t >= 0 ? et : 0xFFu;
    int slot = is_root ? cid : C::RMAX;
    PW_OPAQUE(slot);
    set_par(L, slot, (int)pc);
    ent(L, v) = (Ent)cid;
  }

  // the same with the crossing of the tree edge (v, t) given (odd d); t may
  // also be any vertex of t's region whose id is assigned already
  __device__ static __forceinline__ void vertex3c(const Lane& L, int v, int t, bool crossed, uint32_t ev, int& nR,
                                                  Adj& roots) {
    const uint32_t p = idx(ev);
    const bool is_root = p == (uint32_t)v;
    const uint32_t ep = ent(L, (int)p);  // p < v holds its region id already; a root reads its own entry
    const uint32_t et = ent(L, t < 0 ? 0 : t);
    // ids past the Harnack bound share the spare slot RMAX; finish()
    // rejects such a mask (nR > RMAX) before reading any region data
    const int cid = is_root ? (nR < C::RMAX ? nR : C::RMAX) : (int)ep;
    nR += is_root ? 1 : 0;
    // keep the running count a plain running count (re-associating the
    // chain of increments would hold every vertex's flag in a register)
    PW_OPAQUE(nR);
    const bool hit = C::EVEN ? (is_root && odd_flag(L, (uint32_t)v, ev)) : (crossed && (int)et == cid);
    roots |= hit ? one(cid & (8 * (int)sizeof(Adj) - 1)) : (Adj)0;
    // (a plain running value: between branches the compiler would
    // otherwise keep every vertex's term until the end)
    PW_OPAQUE(roots);
    const uint32_t pc = t >= 0 ? et : 0xFFu;
    int slot = is_root ? cid : C::RMAX;
    PW_OPAQUE(slot);
    set_par(L, slot, (int)pc);
    ent(L, v) = (Ent)cid;
  }

  // A crossed tree edge between vertices a and b (odd d; their regions
  // already assigned) inside one region marks it as the root region, as in
  // vertex3c.
  __device__ static __forceinline__ void hit(const Lane& L, int a, int b, bool crossed, Adj& roots) {
    const uint32_t ra = ent(L, a), rb = ent(L, b);
    roots |= (crossed && ra == rb) ? one((int)ra & (8 * (int)sizeof(Adj) - 1)) : (Adj)0;
    PW_OPAQUE(roots);
  }

  template <class P>
  __device__ static __forceinline__ uint32_t sign_of(P prog, Mask m, int v) {
    const uint32_t rec = prog[v];
    return bit(m, rec & 0x7F) ^ ((rec >> 7) & 1u);
  }

  template <class P>
  __device__ static u128 run(P prog, Mask m, const Lane& L, uint32_t& errs) {
    const P nbr = prog + C::NV;
    const P pairs = prog + C::NV + C::NE;
    clear_side(L);
    // phase 1: components of same-sign vertices
    for (int v = 0; v < C::NV; ++v) {
      const uint32_t rec = prog[v];
      const uint32_t sv = bit(m, rec & 0x7F) ^ ((rec >> 7) & 1u);
      const int nn = (rec >> 8) & 0xFF;
      const int o = rec >> 16;
      uint32_t rv = (uint32_t)v;
      for (int k = 0; k < nn; ++k) {
        const int u = (int)nbr[o + k];
        edge(L, sv, sign_of(prog, m, u), v, rv, u);
      }
      close(L, v, rv);
    }
    // phase 2: regions (antipodal identification)
    for (int t = 0; t < C::NP; ++t) pair(L, pairs[t] & 0xFFFF, pairs[t] >> 16);
    // phase 3: region ids and the region tree
    int nR = 0;
    Adj roots = 0;
    for (int v = 0; v < C::NV; ++v) {
      const int t = v > 0 ? (int)nbr[prog[v] >> 16] : -1;
      vertex3(L, v, t, sign_of(prog, m, v), t >= 0 ? sign_of(prog, m, t) : 0u, nR, roots);
    }
    return finish(L, nR, roots, errs);
  }


  // Phase 4: re-root the region tree at `root` and build the canonical
  // code (AHU) from the leaves up.
  template <class LV>
  __device__ __forceinline__ static u128 finish(const LV& L, int nR, Adj roots, uint32_t& errs) {
    uint32_t err = 0;
    if (roots == 0 || (roots & (roots - 1))) err |= kErrRoot;  // exactly one root region
    if (nR > C::RMAX) err |= C::CAPPED ? kErrOverflow : kErrRegions;
    const int root = roots ? ctz_t(roots) : 0;
    if (err) {
      errs |= err;
      return 0;
    }
    // Every region's parent has a smaller id (region 0 is the top).
    // Re-rooting reverses the parent pointers on the path from `root` to
    // region 0 and leaves every other subtree as it was.
    Adj path = 0;
    {
      int x = root, prev = 0xFF;
      for (int it = 0; x != 0xFF && it < C::RMAX; ++it) {
        const int nx = par(L, x);
        set_par(L, x, prev);
        path |= one(x);
        prev = x;
        x = nx;
      }
      if (x != 0xFF) {
        errs |= kErrTree;
        return 0;
      }
    }
    for (int x = 0; x < nR; ++x) store_adj(L, x, (Adj)0);
    Adj inner = 0;  // regions with at least one child
    for (int x = 0; x < nR; ++x) {
      const int px = par(L, x);
      if (px != 0xFF) {
        store_adj(L, px, load_adj(L, px) | one(x));
        inner |= one(px);
      }
    }
    // Bottom-up order over the regions with children (a leaf is '10' and
    // needs no work): those off the path by decreasing id (all their
    // children have larger ids), then the path from region 0 up to the root
    // (the children of a path region are off the path or the path region
    // done just before it).
    constexpr int AB = 8 * (int)sizeof(Adj);
    const Adj leaves = (nR >= AB ? ~(Adj)0 : (one(nR) - 1)) & ~inner;
    Adj todo = inner & ~path;
    int last = 0xFF;  // the path region done last
    for (int it = 0; it <= C::RMAX; ++it) {
      int y;
      if (todo) {
        y = AB - 1 - clz_t(todo);
        todo &= ~one(y);
      } else {
        y = last == 0xFF ? 0 : par(L, last);
        last = y;
      }
      if ((leaves & one(y)) && y != root) continue;  // a leaf on the path
      const Adj kids = load_adj(L, y);
      Adj rest = kids & ~leaves;
      const int nleaf = popc_t(kids & leaves);
      Code acc = 0;
      int len = 0;
      while (rest) {
        int best = -1;
        Code bkey = 0, bcode = 0;
        Adj t = rest;
        while (t) {
          const int z = ctz_t(t);
          t &= t - 1;
          const Code cz = load_code(L, z);
          const Code kz = cz << clz_t(cz);
          if (best < 0 || kz > bkey) {
            best = z;
            bkey = kz;
            bcode = cz;
          }
        }
        rest &= ~one(best);
        const int lb = (int)(8 * sizeof(Code)) - clz_t(bcode);
        acc = (acc << lb) | bcode;
        len += lb;
      }
      if (nleaf) {
        const Code pat = (~(Code)0 / 3) << 1;  // ...101010
        acc = (acc << (2 * nleaf)) | (pat >> (8 * (int)sizeof(Code) - 2 * nleaf));
        len += 2 * nleaf;
      }
      if (y == root) {
        u128 code = ((u128)1 << len) | (u128)acc;
        if (!C::EVEN) code |= (u128)1 << 127;
        return code;
      }
      store_code(L, y, ((Code)1 << (len + 1)) | (acc << 1));
    }
    errs |= kErrTree;
    return 0;
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

constexpr int kMaxRuns = 4;

// The free bit positions of an enumeration as at most kMaxRuns contiguous
// runs: index bits [src, src+len) go to mask bits [dst, dst+len).  Byte k
// of src / len / dst describes run k.
struct Runs {
  uint32_t n, src, len, dst;
  __host__ __device__ int src_of(int k) const { return (int)((src >> (8 * k)) & 0xFF); }
  __host__ __device__ int len_of(int k) const { return (int)((len >> (8 * k)) & 0xFF); }
  __host__ __device__ int dst_of(int k) const { return (int)((dst >> (8 * k)) & 0xFF); }
  __host__ __device__ void set(int k, int s_, int l_, int d_) {
    const uint32_t m = ~(0xFFu << (8 * k));
    src = (src & m) | ((uint32_t)s_ << (8 * k));
    len = (len & m) | ((uint32_t)l_ << (8 * k));
    dst = (dst & m) | ((uint32_t)d_ << (8 * k));
  }
};

template <typename Mask>
__device__ __forceinline__ Mask deposit_run(uint64_t idx, int src, int len, int dst) {
  const uint64_t keep = len >= 64 ? ~0ull : ((1ull << len) - 1);
  return (Mask)((idx >> src) & keep) << dst;
}

// The run descriptors are passed through an empty asm statement once per
// batch, so the values derived from them are recomputed (a few scalar
// instructions) instead of being held in scalar registers across the
// evaluation.
template <typename Mask>
__device__ __forceinline__ Mask deposit(uint64_t idx, Runs r) {
  PW_OPAQUE_S(r.n);
  PW_OPAQUE_S(r.src);
  PW_OPAQUE_S(r.len);
  PW_OPAQUE_S(r.dst);
  Mask m = deposit_run<Mask>(idx, r.src_of(0), r.len_of(0), r.dst_of(0));
  if (r.n > 1) {  // uniform branch: only class-representative sweeps take it
#pragma unroll
    for (int k = 1; k < kMaxRuns; ++k)
      if (k < (int)r.n) m |= deposit_run<Mask>(idx, r.src_of(k), r.len_of(k), r.dst_of(k));
  }
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

// the table descriptor, read from device memory where it is needed (it is
// not kept in scalar registers across the evaluation)
__device__ __forceinline__ HistDev load_hist(const HistDev* hd) {
  PW_OPAQUE_S(hd);
  return *hd;
}

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

  __device__ __forceinline__ void flush(const HistDev* hd) {
    const HistDev h = load_hist(hd);
    if (!s0.empty()) global_insert(h, s0.lo, s0.hi, s0.cnt, s0.wit);
    if (!s1.empty()) global_insert(h, s1.lo, s1.hi, s1.cnt, s1.wit);
    clear();
  }

  __device__ __forceinline__ void add(uint64_t lo, uint64_t hi, uint64_t k, uint64_t w, int lane,
                                      const HistDev* h) {
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
                                            const HistDev* h) {
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


// ------------------------------------------------------------ kernel bodies
// An evaluator maps (mask, lane memory, error flags) to a scheme code:
// RtEval walks the program in device memory; a kernel generated for one
// triangulation supplies its own straight-line evaluator.

template <int D>
struct RtEval {
  const uint32_t* prog;
  __device__ __forceinline__ u128 operator()(typename Cfg<D>::Mask m, const Lane& L, uint32_t& errs) const {
    return Eval<D>::run(prog, m, L, errs);
  }
};

// this lane's view of its wave's area (lane_words words per lane, the
// parent table at word PAR_BASE)
template <int D, int RCAP = 0>
__device__ __forceinline__ Lane lane_memory(uint32_t* smem, int lane_words) {
  using C = Cfg<D, RCAP>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* base = smem + wave * lane_words * 64;
  char* cb = reinterpret_cast<char*>(base);
  return Lane{base + lane, cb + 4 * C::E_WORDS * lane, cb + C::PAR_BASE * 256 + lane};
}

// the same with the parent table in its own __shared__ array (par: PAR_ROWS
// rows of 64 bytes per wave): the compiler then knows that parent-table
// stores do not alias entry loads and can issue those loads early
template <int D>
__device__ __forceinline__ Lane lane_memory_split(uint32_t* smem, uint8_t* par) {
  using C = Cfg<D>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* base = smem + wave * C::DYN_WORDS * 64;
  return Lane{base + lane, reinterpret_cast<char*>(base) + 4 * C::E_WORDS * lane,
              reinterpret_cast<char*>(par) + wave * C::PAR_ROWS * 64 + lane};
}

// The code of mask i as one 16-byte store (codes must be 16-byte aligned:
// the entry points check it).
struct __attribute__((aligned(16))) Code16 {
  uint64_t lo, hi;
};
__device__ __forceinline__ void store_code(uint64_t* __restrict__ codes, int64_t i, u128 code) {
  *reinterpret_cast<Code16*>(codes + 2 * i) = Code16{(uint64_t)code, (uint64_t)(code >> 64)};
}

// codes of n masks, one per thread, grid-stride
template <int D, class EV>
__device__ __forceinline__ void codes_body(const EV& ev, const void* __restrict__ masks, int64_t n,
                                           uint64_t* __restrict__ codes, uint32_t* __restrict__ errflag,
                                           uint32_t* smem) {
  using C = Cfg<D>;
  __shared__ uint8_t par_rows[C::WAVES * C::PAR_ROWS * 64];
  const Lane L = lane_memory_split<D>(smem, par_rows);
  uint32_t errs = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    const typename C::Mask m = valid ? load_mask<D>(masks, i) : (typename C::Mask)0;
    const u128 code = ev(m, L, errs);
    if (valid) store_code(codes, i, code);
  }
  if (errs) atomicOr(errflag, errs);
}

// histogram of n masks; each wave takes batches of 64 consecutive masks;
// with codes != null the codes are also written (one pass for both)
template <int D, class EV>
__device__ __forceinline__ void hist_body(const EV& ev, const void* __restrict__ masks, int64_t n,
                                          uint64_t index_base, const HistDev* h, uint64_t* __restrict__ codes,
                                          uint32_t* __restrict__ errflag, uint32_t* smem) {
  using C = Cfg<D>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ uint8_t par_rows[C::WAVES * C::PAR_ROWS * 64];
  const Lane L = lane_memory_split<D>(smem, par_rows);
  WaveTable tab;
  tab.clear();
  uint32_t errs = 0;
  const int64_t waves_total = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64; base < n; base += waves_total * 64) {
    const int64_t i = base + lane;
    const bool valid = i < n;
    const typename C::Mask m = valid ? load_mask<D>(masks, i) : (typename C::Mask)0;
    const u128 code = ev(m, L, errs);
    if (codes && valid) store_code(codes, i, code);
    tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, index_base + (uint64_t)i, lane, h);
  }
  tab.flush(h);
  if (errs) atomicOr(errflag, errs);
}

// histogram of the masks generated from indices first .. first+count-1
template <int D, class EV>
__device__ __forceinline__ void enum_body(const EV& ev, uint64_t first, uint64_t count, const Runs& runs,
                                          const HistDev* h, uint32_t* __restrict__ errflag, uint32_t* smem) {
  using C = Cfg<D>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ uint8_t par_rows[C::WAVES * C::PAR_ROWS * 64];
  const Lane L = lane_memory_split<D>(smem, par_rows);
  WaveTable tab;
  tab.clear();
  uint32_t errs = 0;
  const uint64_t waves_total = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64; base < count;
       base += waves_total * 64) {
    const uint64_t k = base + lane;
    const bool valid = k < count;
    const uint64_t idx = first + k;
    const typename C::Mask m = deposit<typename C::Mask>(idx, runs);
    const u128 code = ev(m, L, errs);
    tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, idx, lane, h);
  }
  tab.flush(h);
  if (errs) atomicOr(errflag, errs);
}

// Exhaustive sweep with a shared snapshot.  The index bits 0..5 of an
// enumeration select the lane and bits 6 .. 5+kSnapBits the batch within a
// chunk of 64 << kSnapBits consecutive indices, so inside a chunk only the
// signs of the lattice points those bits map to vary.  ev.snapshot()
// computes, once per chunk, the union-find of the edges between vertices
// whose signs are fixed in the chunk (every lane computes the same one)
// and writes the wave's snapshot row: each such vertex's root, each varying
// vertex's own index; ev.batch() copies the row into the lane's entries,
// adds the edges of the varying vertices and finishes as usual.
constexpr int kSnapBits = 3;

// the mask of the wave's first active lane: for the bits that are equal in
// every lane (the fixed signs of a chunk) a value the compiler keeps in
// scalar registers
// (the builtin returns a signed int: each half is widened as unsigned)
__device__ __forceinline__ uint64_t uniform_mask(uint64_t m) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(m >> 32)) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)m);
}

template <int D, class EV>
__device__ __forceinline__ void enum_snap_body(const EV& ev, uint64_t first, uint64_t count, const Runs& runs,
                                               const HistDev* h, uint32_t* __restrict__ errflag, uint32_t* smem) {
  using C = Cfg<D>;
  constexpr uint64_t CS = 64ull << kSnapBits;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ uint8_t par_rows[C::WAVES * C::PAR_ROWS * 64];
  __shared__ __attribute__((aligned(16))) uint8_t snap_rows[C::WAVES * C::SNAP_BYTES];
  const Lane L = lane_memory_split<D>(smem, par_rows);
  uint8_t* snap = snap_rows + wave * C::SNAP_BYTES;
  WaveTable tab;
  tab.clear();
  uint32_t errs = 0;
  const uint64_t waves_total = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const uint64_t c1 = (first + count - 1) / CS;
  for (uint64_t c = first / CS + (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave; c <= c1; c += waves_total) {
    const uint64_t cbase = c * CS;
    const typename C::Mask mc = deposit<typename C::Mask>(cbase + (uint64_t)lane, runs);
    ev.snapshot(mc, L, snap, lane);
    __builtin_amdgcn_wave_barrier();
    const auto fl = ev.flags(uniform_mask(mc), snap);
    for (int b = 0; b < (1 << kSnapBits); ++b) {
      const uint64_t idx = cbase + (uint64_t)(b * 64 + lane);
      const bool valid = idx >= first && idx - first < count;
      const u128 code = ev.batch(deposit<typename C::Mask>(idx, runs), L, snap, fl, errs);
      tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, idx, lane, h);
    }
    __builtin_amdgcn_wave_barrier();
  }
  tab.flush(h);
  if (errs) atomicOr(errflag, errs);
}

}  // namespace pw
