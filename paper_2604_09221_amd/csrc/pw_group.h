// pw_group.h -- lane groups for the batched launch: G = 2 or 4 lanes of a
// wave evaluate one sign mask together (Alg. 1 of "Fast Isotopy Computation
// for T-Curves", Sec. 2, split over the reflected copies of Sec. 2).
//
// The diamond is the union of the four reflected copies of the
// triangulation, glued along the axes.  Lane q of a group takes one block
// of it -- the quadrant x, y >= 0 reflected by (sx, sy) = (q & 1, q >> 1)
// for G = 4, the half y >= 0 reflected by sy = q for G = 2 -- so every lane
// walks the same block program with its own copy of the mask, flipped by
// the reflection rule of eq. (signs): a point (i, j) of the copy reflected
// by (sx, sy) has the sign of sigma(i, j) times (-1)^(sx i + sy j), i.e. the
// mask XOR a per-lane constant.
//
// Entries: u16, one per (block vertex v, lane q) at group index v * G + q
// (interleaved, so the lanes' entries of one vertex are neighbours).
// Parent indices always point to smaller group indices, so a union-find
// root is the smallest group index of its set, and "every tree parent has
// a smaller index" holds for the spanning tree used in phase 3: a block
// vertex's first earlier neighbour in its own block, or, for a copy of an
// axis point, the same point's copy in a lower block (the glue).
//
// Phases per mask:
//   1 components inside the lane's own block (as for one lane per mask,
//     on the block program; only the lane's own entries are touched);
//   2 glue the copies of the axis points (plain unions: no parity bit is
//     set yet), then the 2d antipodal pairs (with parity for even d).  All
//     lanes of the group run these same steps on the same entries with the
//     same values (lockstep), so the result is that of one lane;
//   3 (a) every lane points each of its vertices straight at its root;
//     (b) in group-index order -- block vertex v, all lanes at once -- a
//     root takes the next region id (the group's roots of this vertex are
//     counted by a ballot), writes it into its entry, and only then are
//     the region ids of the vertex and of its tree parent read (both roots
//     have a group index no larger, so their ids are written already).
//     The region tree is read off that spanning tree exactly as for one
//     lane per mask: the first vertex of a region (its root) hangs below
//     the region of its tree parent; the tree is the region adjacency tree
//     rooted at the region of index 0.  Odd d: a crossed tree edge inside
//     one region marks the root (a glue is never crossed); even d: the
//     odd-cycle flag of phase 2;
//   4 finish() of the one-lane evaluator on the group's region tables, run
//     by all lanes of the group with the same values.
#pragma once
#include "pw_device.h"

namespace pw {

template <int D, int G, int RCAP = 0>
struct GCfg {
  using C = Cfg<D, RCAP>;
  static_assert(G == 2 || G == 4, "lane groups of 2 or 4");
  static_assert(D >= kGroupMinDegree && D <= kDMax, "lane groups serve degrees 8..12");
  static constexpr int NB = group_block_vertices(D, G);
  static constexpr int NEB = group_block_edges(D, G);
  static constexpr int NGL = group_glues(D, G);
  static constexpr int NP = 2 * D;
  static constexpr int NG = 64 / G;             // groups per wave
  static constexpr int NIDX = (NB + 1) * G;     // group indices, with a spare entry per lane (v = NB)
  static_assert(NIDX <= 512, "entry indices fit in 9 bits");
  // a group's entries: GROUP_DW dwords (odd, so that the groups' entries of
  // one vertex start in distinct banks)
  static constexpr int GROUP_DW = ((2 * NIDX + 3) / 4) | 1;
  static constexpr int ENT_DW = GROUP_DW * NG;
  // after phase 3: region word k of group g at dword k * NG + g
  static constexpr int TAB_DW = C::TAIL_WORDS * NG;
  static constexpr int LOW_DW = ENT_DW > TAB_DW ? ENT_DW : TAB_DW;
  // parent table: byte row x (x = 0..RMAX, RMAX the spare) of NG bytes
  static constexpr int PAR_DW = ((C::RMAX + 1) * NG + 3) / 4;
  static constexpr int WAVE_DW = LOW_DW + PAR_DW;
};

// The region tables of one group: word k at w[k * NG], parent byte row x
// at b[x * NG].
template <int NG>
struct GView {
  uint32_t* w;
  uint8_t* b;
  __device__ __forceinline__ uint32_t& word(int k) const { return w[k * NG]; }
  __device__ __forceinline__ uint8_t& prow(int x) const { return b[x * NG]; }
};

template <int D, int G, int RCAP = 0>
struct GroupEval {
  using GC = GCfg<D, G, RCAP>;
  using C = Cfg<D, RCAP>;
  using E = Eval<D, RCAP>;
  using Mask = typename C::Mask;
  using Adj = typename C::Adj;
  using View = GView<GC::NG>;
  static constexpr uint32_t kIdx = 0x1FFu;     // parent index
  static constexpr uint32_t kParity = 0x200u;  // even d: parity to the parent
  static constexpr uint32_t kOdd = 0x400u;     // even d: odd-cycle flag at a root
  static constexpr uint32_t kId = 0x8000u;     // phase 3: a root's entry holds kId | region id
  static constexpr int AB = 8 * (int)sizeof(Adj);

  struct Mem {
    uint16_t* grp;  // the group's entry of index 0
    uint16_t* own;  // this lane's entry of block vertex 0: vertex v at own[v * G]
    View view;
  };

  // lane `lane`'s view of a wave area of GC::WAVE_DW dwords at `wave`
  __device__ __forceinline__ static Mem memory(uint32_t* wave, int lane) {
    const int g = lane / G, q = lane % G;
    uint16_t* grp = reinterpret_cast<uint16_t*>(wave + g * GC::GROUP_DW);
    return Mem{grp, grp + q, View{wave + g, reinterpret_cast<uint8_t*>(wave + GC::LOW_DW) + g}};
  }

  // mask bits of the lattice points (i, j) with i odd (x) or j odd (y)
  static constexpr Mask parity_bits(bool x) {
    Mask r = 0;
    int k = 0;
    for (int j = 0; j <= D; ++j)
      for (int i = 0; i + j <= D; ++i, ++k)
        if ((x ? i : j) & 1) r |= (Mask)1 << k;
    return r;
  }
  // the flip of lane q's copy of the mask (eq. (signs))
  __device__ __forceinline__ static Mask flip(int q) {
    constexpr Mask RX = parity_bits(true), RY = parity_bits(false);
    const int sx = G == 4 ? (q & 1) : 0, sy = G == 4 ? (q >> 1) : q;
    return (sx ? RX : (Mask)0) ^ (sy ? RY : (Mask)0);
  }

  __device__ __forceinline__ static uint32_t bit(Mask m, int p) { return (uint32_t)(m >> p) & 1u; }
  template <class P>
  __device__ __forceinline__ static uint32_t sign(P prog, Mask m, int v) {
    const uint32_t rec = prog[v];
    return bit(m, rec & 0x7F) ^ ((rec >> 7) & 1u);
  }

  // root of index r (entries without parity bits: phases 1 and 2a)
  __device__ __forceinline__ static uint32_t root(const Mem& M, uint32_t r) {
    uint32_t er = M.grp[r];
    while (er != r) {
      r = er;
      PW_OPAQUE(r);
      er = M.grp[r];
    }
    return r;
  }

  // Phase 1 on the lane's own block; m is the lane's flipped mask.  As the
  // one-lane evaluator: a lane whose signs differ stores into v's own
  // entry, which is scratch until v is closed.
  template <class P>
  __device__ static void phase1(P prog, Mask m, const Mem& M, int q) {
    const P nbr = prog + GC::NB;
    for (int v = 0; v < GC::NB; ++v) {
      const uint32_t rec = prog[v];
      const uint32_t sv = bit(m, rec & 0x7F) ^ ((rec >> 7) & 1u);
      const int nn = (rec >> 8) & 0xFF, o = (rec >> 16) & 0xFFF;
      const uint32_t self = (uint32_t)(v * G + q);
      uint32_t rv = self;
      for (int k = 0; k < nn; ++k) {
        const uint32_t nw = nbr[o + k];
        const int u = (int)(nw & 0xFFFF);
        const uint32_t su = bit(m, (nw >> 16) & 0x7F) ^ ((nw >> 23) & 1u);
        const uint32_t r = root(M, M.own[u * G]);
        M.own[u * G] = (uint16_t)r;
        const bool same = su == sv;
        const uint32_t lo = r < rv ? r : rv, hi = r < rv ? rv : r;
        uint32_t w = same ? hi : self;
        PW_OPAQUE(w);
        M.grp[w] = (uint16_t)lo;
        rv = same ? lo : rv;
      }
      M.own[v * G] = (uint16_t)rv;
    }
  }

  __device__ __forceinline__ static uint32_t find_parity(const Mem& M, uint32_t a, uint32_t& er, uint32_t& par) {
    uint32_t r = a;
    er = M.grp[a];
    par = 0;
    while ((er & kIdx) != r) {
      if (C::EVEN) par ^= (er & kParity) ? 1u : 0u;
      r = er & kIdx;
      er = M.grp[r];
    }
    return r;
  }

  // Phase 2: glues, then the antipodal pairs (the same steps in every lane
  // of the group).
  template <class P>
  __device__ static void phase2(P prog, const Mem& M) {
    const P glue = prog + GC::NB + GC::NEB;
    const P pairs = glue + GC::NGL;
    for (int k = 0; k < GC::NGL; ++k) {
      const uint32_t ra = root(M, glue[k] & 0xFFFF), rb = root(M, glue[k] >> 16);
      const uint32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
      M.grp[hi] = (uint16_t)lo;  // a no-op rewrite when ra == rb
    }
    for (int k = 0; k < GC::NP; ++k) {
      uint32_t ea, eb, pa, pb;
      const uint32_t ra = find_parity(M, pairs[k] & 0xFFFF, ea, pa);
      const uint32_t rb = find_parity(M, pairs[k] >> 16, eb, pb);
      if (ra == rb) {
        if (C::EVEN && pa == pb) M.grp[ra] = (uint16_t)(ea | kOdd);
      } else {
        const bool a_lo = ra < rb;
        const uint32_t lo = a_lo ? ra : rb, hi = a_lo ? rb : ra;
        const uint32_t elo = a_lo ? ea : eb, ehi = a_lo ? eb : ea;
        const uint32_t par = C::EVEN ? ((pa ^ pb ^ 1u) ? kParity : 0u) : 0u;
        M.grp[hi] = (uint16_t)(par | lo);
        if (C::EVEN && (ehi & kOdd)) M.grp[lo] = (uint16_t)(elo | kOdd);
      }
    }
  }

  // Phase 3a: each of the lane's vertices points straight at its root
  // (a root keeps its entry and its odd-cycle flag).  Other lanes may walk
  // through these entries meanwhile; they see the old parent or the root,
  // both ancestors.
  __device__ static void phase3a(const Mem& M, int q) {
    for (int v = 0; v < GC::NB; ++v) {
      const uint32_t self = (uint32_t)(v * G + q);
      const uint32_t e = M.own[v * G];
      uint32_t r = e & kIdx;
      uint32_t er = M.grp[r];
      while ((er & kIdx) != r) {
        r = er & kIdx;
        PW_OPAQUE(r);
        er = M.grp[r];
      }
      M.own[v * G] = (uint16_t)(r == self ? e : r);
    }
  }

  // Phase 3b, vertex v, first half: is v a root (its entry, after 3a)?
  __device__ __forceinline__ static bool p3_is_root(const Mem& M, int v, int q, uint32_t& ev) {
    ev = M.own[v * G];
    return (ev & kIdx) == (uint32_t)(v * G + q);
  }
  // ... a root writes its region id (a non-root writes its spare entry)
  __device__ __forceinline__ static void p3_write(const Mem& M, int v, bool is_root, int cid) {
    int slot = is_root ? v : GC::NB;
    PW_OPAQUE(slot);
    M.own[slot * G] = (uint16_t)(kId | (uint32_t)cid);
  }
  // region id of group index x (after the writes of every index <= x)
  __device__ __forceinline__ static uint32_t region(const Mem& M, uint32_t x) {
    const uint32_t e = M.grp[x];
    const uint32_t e2 = M.grp[e & kIdx];  // the root's entry (unused when x is a root)
    return ((e & kId) ? e : e2) & 0xFFu;
  }
  // ... second half: the region tree edge of a root, the root region
  // marks.  cid: v's id if v is a root (capped at RMAX).
  template <class P>
  __device__ __forceinline__ static void p3_link(P prog, Mask m, const Mem& M, int v, int q,
                                                 bool is_root, uint32_t ev, int cid, Adj& roots) {
    const uint32_t rec = prog[v];
    const int sx = G == 4 ? (q & 1) : 0, sy = G == 4 ? (q >> 1) : q;
    const bool gx = sx && ((rec >> 28) & 1u), gy = sy && ((rec >> 29) & 1u);
    const bool glued = gx || gy;
    const bool has_t = v > 0 || q > 0;
    const uint32_t tw = v > 0 ? prog[GC::NB + ((rec >> 16) & 0xFFF)] : 0u;
    const int t_loc = (int)(tw & 0xFFFF);
    const uint32_t t_idx = glued ? (uint32_t)(v * G + q - (gx ? 1 : (G == 4 ? 2 : 1))) : (uint32_t)(t_loc * G + q);
    const uint32_t rt = region(M, has_t ? t_idx : 0u);
    const uint32_t rid = is_root ? (uint32_t)cid : (M.grp[ev & kIdx] & 0xFFu);
    int slot = is_root ? cid : C::RMAX;
    PW_OPAQUE(slot);
    E::set_par(M.view, slot, has_t ? (int)rt : 0xFF);
    bool hit;
    if constexpr (C::EVEN) {
      hit = is_root && (ev & kOdd);
    } else {
      const bool crossed = has_t && !glued && sign(prog, m, v) != (bit(m, (tw >> 16) & 0x7F) ^ ((tw >> 23) & 1u));
      hit = crossed && rid == rt;
    }
    roots |= hit ? E::one((int)rid & (AB - 1)) : (Adj)0;
    PW_OPAQUE(roots);
  }

  __device__ __forceinline__ static Adj group_or(Adj x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)((uint64_t)x >> 32);
    for (int s = 1; s < G; s <<= 1) {
      lo |= (uint32_t)__shfl_xor((int)lo, s, 64);
      if (sizeof(Adj) > 4) hi |= (uint32_t)__shfl_xor((int)hi, s, 64);
    }
    return (Adj)((uint64_t)lo | ((uint64_t)hi << 32));
  }

  // The whole evaluation; m is the lane's flipped mask.  Every lane of the
  // group returns the same code and error flags.
  template <class P>
  __device__ static u128 run(P prog, Mask m, const Mem& M, int lane, int q,
                             uint32_t& errs) {
    phase1(prog, m, M, q);
    PW_FENCE();
    phase2(prog, M);
    PW_FENCE();
    phase3a(M, q);
    PW_FENCE();
    int nR = 0;
    Adj roots = 0;
    const int gsh = lane & ~(G - 1);
    for (int v = 0; v < GC::NB; ++v) {
      uint32_t ev;
      const bool is_root = p3_is_root(M, v, q, ev);
      const uint32_t gb = (uint32_t)(__ballot(is_root) >> gsh) & ((1u << G) - 1u);
      const int id = nR + __popc(gb & ((1u << q) - 1u));
      nR += __popc(gb);
      // ids past the table size share the spare slot RMAX; finish()
      // rejects such a mask (nR > RMAX) before reading any region data
      const int cid = id < C::RMAX ? id : C::RMAX;
      p3_write(M, v, is_root, cid);
      PW_FENCE();
      p3_link(prog, m, M, v, q, is_root, ev, cid, roots);
      PW_FENCE();
    }
    roots = group_or(roots);
    return E::finish(M.view, nR, roots, errs);
  }
};

}  // namespace pw
