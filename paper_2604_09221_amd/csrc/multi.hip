// multi.hip -- persistent launches over many triangulations of uneven
// degree (Sec. 3: the second search mode checks many triangulations against
// sign distributions; the paper names kernel dispatch and histogram
// aggregation as the costs at scale).
//
// The host cuts every triangulation's mask list into chunks, groups the
// chunks by LDS class (degrees whose per-wave areas allow the same number
// of resident waves per CU), orders each group by decreasing cost (chunk
// length x |E(T<>)|, longest processing time first) and uploads them.  Per
// class one persistent launch, its LDS sized for the class's largest
// degree: resident waves take chunks from an atomic ticket counter until
// none is left; each chunk is evaluated with the degree-specialised Eval<D>
// and aggregated in the wave's register table, which is flushed to that
// triangulation's histogram when the chunk ends.  The ticket counter only
// grows, so no launch ever has to reset it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cstdint>
#include <cstring>
#include <vector>

#include "patchwork.h"
#include "pw_device.h"
#include "pw_group.h"
#include "pw_host.h"

namespace pw {

struct TriDesc {
  const uint32_t* prog;
  const uint32_t* gprog[2];  // group programs for 2 and 4 lanes per mask (degrees 8..12), else null
  uint32_t* err;
  const HistDev* hist;
  int32_t d;
  int32_t use_hist;
};

struct Item {
  int32_t tri;
  int32_t pad;
  int64_t begin;  // first mask (global index into the mask array)
  int64_t count;
};

// Degrees >= 10 use phase-4 tables capped at 32 regions (about half the
// LDS of the full tables at d = 12, so more waves fit per CU); a mask with
// more regions is put on an overflow list and evaluated again, with the
// full tables, by k_multi_big after the persistent launch.
constexpr int multi_cap(int d) { return d >= 10 ? 32 : 0; }

struct Overflow {
  uint64_t* list;              // (triangulation, global mask index) pairs
  unsigned long long* n;       // entries claimed (may exceed cap)
  unsigned long long cap;
};

template <int D>
__device__ __forceinline__ void run_item(const TriDesc& t, const Item& w, const uint64_t* __restrict__ masks,
                                         uint64_t* __restrict__ codes, uint32_t* smem, int lane_words, int lane,
                                         const Overflow& ov) {
  constexpr int RC = multi_cap(D);
  using C = Cfg<D, RC>;
  const Lane L = lane_memory<D, RC>(smem, lane_words);
  uint32_t errs = 0;
  WaveTable tab;
  tab.clear();
  for (int64_t base = 0; base < w.count; base += 64) {
    const int64_t i = w.begin + base + lane;
    bool valid = base + lane < w.count;
    typename C::Mask m = 0;
    if (valid) {
      if constexpr (sizeof(typename C::Mask) == 8) {
        m = masks[2 * i];
      } else {
        m = ((u128)masks[2 * i + 1] << 64) | (u128)masks[2 * i];
      }
    }
    uint32_t e = 0;
    const u128 code = Eval<D, RC>::run(const_prog(t.prog), m, L, e);
    if (C::CAPPED && (e & kErrOverflow) && valid) {
      const unsigned long long slot = atomicAdd(ov.n, 1ull);
      if (slot < ov.cap) {
        ov.list[2 * slot] = (uint64_t)w.tri;
        ov.list[2 * slot + 1] = (uint64_t)i;
      }
      valid = false;  // counted and written by k_multi_big
    }
    errs |= e & ~kErrOverflow;
    if (codes && valid) store_code(codes, i, code);
    if (t.use_hist) tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, (uint64_t)i, lane, t.hist);
  }
  if (t.use_hist) tab.flush(t.hist);
  if (errs) atomicOr(t.err, errs);
}

__global__ __launch_bounds__(256) void k_multi(const TriDesc* __restrict__ tris, const Item* __restrict__ items,
                                               int64_t n_items, unsigned long long* __restrict__ ticket,
                                               unsigned long long base, const uint64_t* __restrict__ masks,
                                               uint64_t* __restrict__ codes, int lane_words, Overflow ov) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  while (true) {
    unsigned long long tk = 0;
    if (lane == 0) tk = atomicAdd(ticket, 1ull);
    // (the builtin returns a signed int: both halves are widened as unsigned)
    tk = (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)tk) |
         ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(tk >> 32)) << 32);
    const int64_t it = (int64_t)(tk - base);
    if (it >= n_items) break;
    const Item w = items[it];
    const TriDesc t = tris[w.tri];
    switch (t.d) {
      case 1: run_item<1>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 2: run_item<2>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 3: run_item<3>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 4: run_item<4>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 5: run_item<5>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 6: run_item<6>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 7: run_item<7>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 8: run_item<8>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 9: run_item<9>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 10: run_item<10>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 11: run_item<11>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      case 12: run_item<12>(t, w, masks, codes, smem, lane_words, lane, ov); break;
      default: break;
    }
  }
}

// The same with G lanes per mask (pw_group.h): the wave takes 64 / G masks
// per batch; lane q of group g evaluates block q of mask begin + base + g,
// and lane 0 of the group writes its code and counts it.
template <int D, int G>
__device__ __forceinline__ void run_item_g(const TriDesc& t, const Item& w, const uint64_t* __restrict__ masks,
                                           uint64_t* __restrict__ codes, uint32_t* wave, int lane,
                                           const Overflow& ov) {
  constexpr int RC = multi_cap(D);
  using GE = GroupEval<D, G, RC>;
  using C = typename GE::C;
  constexpr int NG = GE::GC::NG;
  const typename GE::Mem M = GE::memory(wave, lane);
  const int q = lane % G, g = lane / G;
  const typename C::Mask fl = GE::flip(q);
  const prog_ptr prog = const_prog(t.gprog[G == 4 ? 1 : 0]);
  uint32_t errs = 0;
  WaveTable tab;
  tab.clear();
  for (int64_t base = 0; base < w.count; base += NG) {
    const int64_t i = w.begin + base + g;
    bool valid = base + g < w.count;
    typename C::Mask m = 0;
    if (valid) {
      if constexpr (sizeof(typename C::Mask) == 8) {
        m = masks[2 * i];
      } else {
        m = ((u128)masks[2 * i + 1] << 64) | (u128)masks[2 * i];
      }
    }
    uint32_t e = 0;
    const u128 code = GE::run(prog, m ^ fl, M, lane, q, e);
    valid = valid && q == 0;
    if (C::CAPPED && (e & kErrOverflow) && valid) {
      const unsigned long long slot = atomicAdd(ov.n, 1ull);
      if (slot < ov.cap) {
        ov.list[2 * slot] = (uint64_t)w.tri;
        ov.list[2 * slot + 1] = (uint64_t)i;
      }
      valid = false;  // counted and written by k_multi_big
    }
    errs |= e & ~kErrOverflow;
    if (codes && valid) store_code(codes, i, code);
    // (valid lanes hold increasing indices: the lowest lane of a match has
    // the smallest witness)
    if (t.use_hist) tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, (uint64_t)i, lane, t.hist);
  }
  if (t.use_hist) tab.flush(t.hist);
  if (errs) atomicOr(t.err, errs);
}

// k_multi with G lanes per mask; wave_dw dwords of LDS per wave.  Only
// degrees 8..12 are given to it.
template <int G>
__global__ __launch_bounds__(256) void k_multi_g(const TriDesc* __restrict__ tris, const Item* __restrict__ items,
                                                 int64_t n_items, unsigned long long* __restrict__ ticket,
                                                 unsigned long long base, const uint64_t* __restrict__ masks,
                                                 uint64_t* __restrict__ codes, int wave_dw, Overflow ov) {
  extern __shared__ uint32_t smem[];
  const int lane = threadIdx.x & 63;
  uint32_t* wave = smem + (threadIdx.x >> 6) * wave_dw;
  while (true) {
    unsigned long long tk = 0;
    if (lane == 0) tk = atomicAdd(ticket, 1ull);
    tk = (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)tk) |
         ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(tk >> 32)) << 32);
    const int64_t it = (int64_t)(tk - base);
    if (it >= n_items) break;
    const Item w = items[it];
    const TriDesc t = tris[w.tri];
    switch (t.d) {
      case 8: run_item_g<8, G>(t, w, masks, codes, wave, lane, ov); break;
      case 9: run_item_g<9, G>(t, w, masks, codes, wave, lane, ov); break;
      case 10: run_item_g<10, G>(t, w, masks, codes, wave, lane, ov); break;
      case 11: run_item_g<11, G>(t, w, masks, codes, wave, lane, ov); break;
      case 12: run_item_g<12, G>(t, w, masks, codes, wave, lane, ov); break;
      default: break;
    }
  }
}

template __global__ void k_multi_g<2>(const TriDesc*, const Item*, int64_t, unsigned long long*, unsigned long long,
                                      const uint64_t*, uint64_t*, int, Overflow);
template __global__ void k_multi_g<4>(const TriDesc*, const Item*, int64_t, unsigned long long*, unsigned long long,
                                      const uint64_t*, uint64_t*, int, Overflow);

// One overflow entry per lane, full phase-4 tables (Cfg<D>).
template <int D>
__device__ __forceinline__ void run_big(const TriDesc& t, int64_t i, const uint64_t* __restrict__ masks,
                                        uint64_t* __restrict__ codes, uint32_t* smem) {
  using C = Cfg<D>;
  const Lane L = lane_memory<D>(smem, Cfg<12>::LANE_WORDS);
  typename C::Mask m;
  if constexpr (sizeof(typename C::Mask) == 8) {
    m = masks[2 * i];
  } else {
    m = ((u128)masks[2 * i + 1] << 64) | (u128)masks[2 * i];
  }
  uint32_t e = 0;
  const u128 code = Eval<D>::run(const_prog(t.prog), m, L, e);
  if (e) atomicOr(t.err, e);
  if (codes) store_code(codes, i, code);
  // (the descriptor differs between lanes here: a plain vector load)
  if (t.use_hist && code != 0) global_insert(*t.hist, (uint64_t)code, (uint64_t)(code >> 64), 1, (uint64_t)i);
}

__global__ __launch_bounds__(64) void k_multi_big(const TriDesc* __restrict__ tris, const uint64_t* __restrict__ list,
                                                  int64_t n, const uint64_t* __restrict__ masks,
                                                  uint64_t* __restrict__ codes) {
  extern __shared__ uint32_t smem[];
  for (int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 64) {
    const TriDesc t = tris[list[2 * k]];
    const int64_t i = (int64_t)list[2 * k + 1];
    switch (t.d) {
      case 10: run_big<10>(t, i, masks, codes, smem); break;
      case 11: run_big<11>(t, i, masks, codes, smem); break;
      case 12: run_big<12>(t, i, masks, codes, smem); break;
      default: break;
    }
  }
}

// LDS dwords per wave of k_multi_g<G> at degree d
template <int G>
int group_wave_dw(int d) {
  switch (d) {
    case 8: return GCfg<8, G, multi_cap(8)>::WAVE_DW;
    case 9: return GCfg<9, G, multi_cap(9)>::WAVE_DW;
    case 10: return GCfg<10, G, multi_cap(10)>::WAVE_DW;
    case 11: return GCfg<11, G, multi_cap(11)>::WAVE_DW;
    case 12: return GCfg<12, G, multi_cap(12)>::WAVE_DW;
    default: return 0;
  }
}

int lane_words_for(int d) {
  switch (d) {
    case 1: return Cfg<1>::LANE_WORDS;
    case 2: return Cfg<2>::LANE_WORDS;
    case 3: return Cfg<3>::LANE_WORDS;
    case 4: return Cfg<4>::LANE_WORDS;
    case 5: return Cfg<5>::LANE_WORDS;
    case 6: return Cfg<6>::LANE_WORDS;
    case 7: return Cfg<7>::LANE_WORDS;
    case 8: return Cfg<8>::LANE_WORDS;
    case 9: return Cfg<9>::LANE_WORDS;
    case 10: return Cfg<10, multi_cap(10)>::LANE_WORDS;
    case 11: return Cfg<11, multi_cap(11)>::LANE_WORDS;
    case 12: return Cfg<12, multi_cap(12)>::LANE_WORDS;
    default: return 0;
  }
}

// Device buffers reused across calls (grown on demand, freed at exit).
struct MultiScratch {
  std::mutex mu;
  TriDesc* d_tris = nullptr;
  size_t tri_cap = 0;
  Item* d_items = nullptr;
  size_t item_cap = 0;
  unsigned long long* d_ticket = nullptr;
  unsigned long long issued = 0;  // tickets handed out by earlier launches
  uint64_t* d_over = nullptr;     // overflow list (kOverflowCap pairs)
  unsigned long long* d_over_n = nullptr;
};

constexpr unsigned long long kOverflowCap = 1ull << 20;

MultiScratch& scratch_for_multi() {
  static MultiScratch s;
  return s;
}

// Fixed device array of patchwork_scheme_batch_multi_noalloc: the ticket
// counter and the overflow count, the descriptor table, the work-item table
// and the overflow list of one call, at the offsets below.  Every GPU the
// library runs on holds its own copy until the process ends.  Host code
// never passes `scratch` itself to a kernel (in host code the name is a
// stand-in, not a device address): it uses the address returned for the
// current device by hipGetSymbolAddress.
constexpr size_t kNaTicket = 0;                                         // u64
constexpr size_t kNaOverN = 8;                                          // u64
constexpr size_t kNaTris = 256;                                         // TriDesc[PW_NOALLOC_MAX_TRIS]
constexpr size_t kNaItems = kNaTris + sizeof(TriDesc) * PW_NOALLOC_MAX_TRIS;  // Item[PW_NOALLOC_MAX_ITEMS]
constexpr size_t kNaOver = kNaItems + sizeof(Item) * PW_NOALLOC_MAX_ITEMS;    // u64[2 * PW_NOALLOC_MAX_OVERFLOW]
constexpr size_t kNaBytes = kNaOver + sizeof(uint64_t) * 2 * PW_NOALLOC_MAX_OVERFLOW;
static_assert(kNaItems % 256 == 0 && kNaOver % 256 == 0, "scratch sections stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

__global__ void k_clear_u64(uint64_t* p, int n) {
  const int i = (int)threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace pw

using namespace pw;

namespace {

// The host part of a call: descriptors, work items and LDS classes.
struct MultiPlan {
  std::vector<TriDesc> desc;
  std::vector<Item> items;  // grouped by class (in launch order), longest first within a class
  struct Shape {
    int wave_dw, wpb, per_cu, group;  // LDS dwords per wave, waves per block, blocks per CU, lanes per mask
  };
  std::vector<Shape> cls;
  std::vector<int> order;  // classes in launch order
  int cls_of_deg[13];
};

// Device buffers one call runs on: descriptor and item tables, the ticket
// counter and the overflow list.
struct MultiBuffers {
  TriDesc* tris;
  Item* items;
  unsigned long long* ticket;
  unsigned long long* issued;  // host copy: tickets handed out by earlier launches on `ticket`
  uint64_t* over;
  unsigned long long* over_n;
  unsigned long long over_cap;
};

pw_status plan_multi(const pw_tri_t* tris, int32_t n_tris, const void* d_masks, const int64_t* offsets,
                     const pw_hist_t* hists, uint64_t* d_codes, const pw_multi_config* cfg, MultiPlan& P) {
  if (!tris || n_tris < 0 || !offsets) return set_err(PW_ERR_ARG, "null or negative argument");
  if (n_tris == 0) return PW_OK;
  if (!hists && !d_codes) return set_err(PW_ERR_ARG, "need histograms, codes or both");
  if ((uintptr_t)d_codes & 15) return set_err(PW_ERR_ARG, "d_codes must be 16-byte aligned");
  pw_multi_config c = {4096, 1, 0, PW_MULTI_DEFAULT_LANE_GROUPS};
  if (cfg) c = *cfg;
  if (c.chunk < 64 || c.chunk > (1 << 24) || c.waves_per_block < 1 || c.waves_per_block > 4 ||
      c.blocks_per_cu < 0 || c.blocks_per_cu > 32)
    return set_err(PW_ERR_ARG, "bad multi config (chunk %d, waves %d, blocks/CU %d)", c.chunk, c.waves_per_block,
                   c.blocks_per_cu);
  for (int d = 0; d <= 15; ++d) {
    const uint32_t code = (c.lane_groups >> (2 * d)) & 3u;
    if (code == 3 || (code != 0 && (d < kGroupMinDegree || d > kDMax)))
      return set_err(PW_ERR_ARG, "bad lane group code %u for degree %d (lane_groups 0x%x)", code, d, c.lane_groups);
  }
  std::vector<TriDesc>& desc = P.desc;
  std::vector<Item>& items = P.items;
  desc.assign(n_tris, TriDesc{});
  items.clear();
  for (int t = 0; t < n_tris; ++t) {
    if (!tris[t]) return set_err(PW_ERR_ARG, "null triangulation %d", t);
    if (offsets[t + 1] < offsets[t] || offsets[t] < 0) return set_err(PW_ERR_ARG, "offsets must not decrease");
    if (hists && !hists[t]) return set_err(PW_ERR_ARG, "null histogram %d", t);
    const int d = tris[t]->prog.d;
    desc[t].prog = tris[t]->d_prog;
    desc[t].gprog[0] = tris[t]->d_gprog[0];
    desc[t].gprog[1] = tris[t]->d_gprog[1];
    desc[t].err = tris[t]->d_err;
    desc[t].hist = hists ? hists[t]->d_dev : nullptr;
    desc[t].d = d;
    desc[t].use_hist = hists ? 1 : 0;
    for (int64_t b = offsets[t]; b < offsets[t + 1]; b += c.chunk)
      items.push_back(Item{t, 0, b, std::min<int64_t>(c.chunk, offsets[t + 1] - b)});
  }
  if (items.empty()) return PW_OK;
  if (!d_masks) return set_err(PW_ERR_ARG, "null mask buffer");
  const void* kern[3] = {reinterpret_cast<const void*>(&k_multi), reinterpret_cast<const void*>(&k_multi_g<2>),
                         reinterpret_cast<const void*>(&k_multi_g<4>)};
  static const hipError_t attr = [&] {
    hipError_t e = hipSuccess;
    for (const void* k : kern)
      if (e == hipSuccess) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    return e;
  }();
  if (attr != hipSuccess) {
    (void)hipGetLastError();
    return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
  }
  // One launch per LDS class.  A wave's area has to hold the largest degree
  // it may meet, so a single launch would give every wave the area of the
  // largest degree present (3 waves per CU at d = 12).  Degrees whose own
  // areas allow the same number of resident blocks per CU (LDS, registers
  // and the configured cap) share a launch sized for the largest of them;
  // the launches follow each other on the stream.  A degree evaluated
  // with lane groups (G lanes per mask) uses the kernel for G, so its
  // class holds only degrees with the same G.
  using Shape = MultiPlan::Shape;
  auto shape_for = [&](int wave_dw, int group) {
    Shape s{wave_dw, c.waves_per_block, 1, group};
    while (s.wpb > 1 && (size_t)wave_dw * 4 * s.wpb > 160 * 1024) --s.wpb;
    const size_t lds = (size_t)wave_dw * 4 * s.wpb;
    int per_cu = (int)((160 * 1024) / lds);
    int by_regs = 0;  // resident blocks allowed by the register budget alone
    const void* k = kern[group == 1 ? 0 : (group == 2 ? 1 : 2)];
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&by_regs, k, 64 * s.wpb, 0) == hipSuccess) {
      if (by_regs > 0) per_cu = std::min(per_cu, by_regs);
    } else {
      (void)hipGetLastError();
    }
    if (c.blocks_per_cu > 0) per_cu = std::min(per_cu, c.blocks_per_cu);
    s.per_cu = std::max(1, std::min(per_cu, 32 / s.wpb));
    return s;
  };
  std::vector<Shape>& cls = P.cls;
  cls.clear();
  for (int d = 0; d <= 12; ++d) P.cls_of_deg[d] = -1;
  for (const TriDesc& t : desc) {
    if (t.d < 1 || t.d > 12) return set_err(PW_ERR_ARG, "degree %d outside 1..12", t.d);
    if (P.cls_of_deg[t.d] >= 0) continue;
    const uint32_t code = (c.lane_groups >> (2 * t.d)) & 3u;
    const int group = code == 0 ? 1 : (code == 1 ? 2 : 4);
    if (group > 1 && !t.gprog[group == 2 ? 0 : 1])
      return set_err(PW_ERR_INTERNAL, "triangulation of degree %d has no group program", t.d);
    const int wave_dw = group == 1 ? 64 * lane_words_for(t.d)
                                   : (group == 2 ? group_wave_dw<2>(t.d) : group_wave_dw<4>(t.d));
    const Shape s = shape_for(wave_dw, group);
    if ((size_t)s.wave_dw * 4 * s.wpb > 160 * 1024)
      return set_err(PW_ERR_ARG, "block needs %zu bytes of LDS", (size_t)s.wave_dw * 4 * s.wpb);
    int k = 0;
    while (k < (int)cls.size() && (cls[k].per_cu != s.per_cu || cls[k].wpb != s.wpb || cls[k].group != s.group)) ++k;
    if (k == (int)cls.size()) cls.push_back(s);
    cls[k].wave_dw = std::max(cls[k].wave_dw, s.wave_dw);
    P.cls_of_deg[t.d] = k;
  }
  // longest processing time first within a class: cost ~ chunk length x
  // diamond edges; classes with the largest areas go first
  std::vector<int>& order = P.order;
  order.resize(cls.size());
  for (size_t k = 0; k < cls.size(); ++k) order[k] = (int)k;
  // (per mask: a wave's area times G over 64 masks)
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return (int64_t)cls[a].wave_dw * cls[a].group > (int64_t)cls[b].wave_dw * cls[b].group;
  });
  std::vector<int> rank(cls.size());
  for (size_t k = 0; k < order.size(); ++k) rank[order[k]] = (int)k;
  std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) {
    const int ra = rank[P.cls_of_deg[desc[a.tri].d]], rb = rank[P.cls_of_deg[desc[b.tri].d]];
    if (ra != rb) return ra < rb;
    const int64_t ca = a.count * n_diamond_edges(desc[a.tri].d), cb = b.count * n_diamond_edges(desc[b.tri].d);
    return ca > cb;
  });
  return PW_OK;
}

// Uploads the plan's tables into B, runs one persistent launch per class,
// then the overflow kernel; returns after the stream has finished.
pw_status run_multi(const MultiPlan& P, MultiBuffers& B, const void* d_masks, uint64_t* d_codes,
                    hipStream_t stream) {
  const std::vector<TriDesc>& desc = P.desc;
  const std::vector<Item>& items = P.items;
  // the descriptor and item tables are reused by the next call: the copies
  // finish before the call returns (it synchronises the stream)
  PW_HIP(hipMemcpyAsync(B.tris, desc.data(), sizeof(TriDesc) * desc.size(), hipMemcpyHostToDevice, stream));
  PW_HIP(hipMemcpyAsync(B.items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice, stream));
  const Overflow ov{B.over, B.over_n, B.over_cap};
  size_t first = 0;
  for (const int k : P.order) {
    size_t last = first;
    while (last < items.size() && P.cls_of_deg[desc[items[last].tri].d] == k) ++last;
    const int64_t n = (int64_t)(last - first);
    if (n == 0) continue;  // a class whose triangulations have no masks
    const MultiPlan::Shape& s = P.cls[k];
    const size_t lds = (size_t)s.wave_dw * 4 * s.wpb;
    const int64_t blocks = std::min<int64_t>((int64_t)cu_count() * s.per_cu, (n + s.wpb - 1) / s.wpb);
    const unsigned long long base = *B.issued;
    // every wave takes one ticket past the end of its launch before it stops
    *B.issued += (unsigned long long)n + (unsigned long long)blocks * s.wpb;
    const uint64_t* masks = static_cast<const uint64_t*>(d_masks);
    if (s.group == 1)
      hipLaunchKernelGGL(k_multi, dim3((unsigned)blocks), dim3(64 * s.wpb), lds, stream, B.tris, B.items + first, n,
                         B.ticket, base, masks, d_codes, s.wave_dw / 64, ov);
    else if (s.group == 2)
      hipLaunchKernelGGL(k_multi_g<2>, dim3((unsigned)blocks), dim3(64 * s.wpb), lds, stream, B.tris,
                         B.items + first, n, B.ticket, base, masks, d_codes, s.wave_dw, ov);
    else
      hipLaunchKernelGGL(k_multi_g<4>, dim3((unsigned)blocks), dim3(64 * s.wpb), lds, stream, B.tris,
                         B.items + first, n, B.ticket, base, masks, d_codes, s.wave_dw, ov);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) {
      *B.issued = base;  // a launch that failed took no tickets
      return set_err(PW_ERR_HIP, "k_multi launch: %s (code %d)", hipGetErrorString(le), (int)le);
    }
    first = last;
  }
  unsigned long long n_over = 0;
  PW_HIP(hipMemcpyAsync(&n_over, B.over_n, sizeof n_over, hipMemcpyDeviceToHost, stream));
  PW_HIP(hipStreamSynchronize(stream));
  if (n_over > B.over_cap)
    return set_err(PW_ERR_INTERNAL, "%llu masks have more than 31 ovals (at most %llu per call): split the call",
                   n_over, B.over_cap);
  if (n_over > 0) {
    const size_t big_lds = (size_t)Cfg<12>::LANE_WORDS * 4 * 64;
    static const hipError_t attr_big = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_multi_big),
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr_big != hipSuccess) {
      (void)hipGetLastError();
      return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr_big), (int)attr_big);
    }
    const int64_t nb = std::min<int64_t>(((int64_t)n_over + 63) / 64, (int64_t)cu_count());
    hipLaunchKernelGGL(k_multi_big, dim3((unsigned)nb), dim3(64), big_lds, stream, B.tris, B.over, (int64_t)n_over,
                       static_cast<const uint64_t*>(d_masks), d_codes);
    PW_HIP(hipGetLastError());
    PW_HIP(hipStreamSynchronize(stream));
  }
  return PW_OK;
}

}  // namespace

extern "C" pw_status patchwork_scheme_batch_multi(const pw_tri_t* tris, int32_t n_tris, const void* d_masks,
                                                  const int64_t* offsets, const pw_hist_t* hists,
                                                  uint64_t* d_codes, const pw_multi_config* cfg,
                                                  hipStream_t stream) {
  MultiPlan P;
  const pw_status st = plan_multi(tris, n_tris, d_masks, offsets, hists, d_codes, cfg, P);
  if (st != PW_OK || P.items.empty()) return st;
  MultiScratch& S = scratch_for_multi();
  std::lock_guard<std::mutex> lock(S.mu);
  if (S.tri_cap < P.desc.size()) {
    if (S.d_tris) (void)hipFree(S.d_tris);
    S.d_tris = nullptr;
    PW_HIP(hipMalloc(&S.d_tris, sizeof(TriDesc) * P.desc.size()));
    S.tri_cap = P.desc.size();
  }
  if (S.item_cap < P.items.size()) {
    if (S.d_items) (void)hipFree(S.d_items);
    S.d_items = nullptr;
    PW_HIP(hipMalloc(&S.d_items, sizeof(Item) * P.items.size()));
    S.item_cap = P.items.size();
  }
  if (!S.d_ticket) {
    PW_HIP(hipMalloc(&S.d_ticket, sizeof(unsigned long long)));
    PW_HIP(hipMemset(S.d_ticket, 0, sizeof(unsigned long long)));
    S.issued = 0;
  }
  if (!S.d_over) {
    PW_HIP(hipMalloc(&S.d_over, sizeof(uint64_t) * 2 * kOverflowCap));
    PW_HIP(hipMalloc(&S.d_over_n, sizeof(unsigned long long)));
  }
  PW_HIP(hipMemsetAsync(S.d_over_n, 0, sizeof(unsigned long long), stream));
  MultiBuffers B{S.d_tris, S.d_items, S.d_ticket, &S.issued, S.d_over, S.d_over_n, kOverflowCap};
  return run_multi(P, B, d_masks, d_codes, stream);
}

namespace {

constexpr int kNaMaxDevices = 64;

// Address of `scratch` on each device, looked up once per device (with that
// device current) on the first call there.
struct NoallocState {
  std::mutex mu;
  unsigned char* ptr[kNaMaxDevices] = {};
};

NoallocState& noalloc_state() {
  static NoallocState s;
  return s;
}

}  // namespace

extern "C" pw_status patchwork_scheme_batch_multi_noalloc(const pw_tri_t* tris, int32_t n_tris,
                                                          const void* d_masks, const int64_t* offsets,
                                                          const pw_hist_t* hists, uint64_t* d_codes,
                                                          const pw_multi_config* cfg, hipStream_t stream) {
  if (n_tris > PW_NOALLOC_MAX_TRIS)
    return set_err(PW_ERR_ARG, "%d triangulations: the allocation-free call takes at most %d", n_tris,
                   PW_NOALLOC_MAX_TRIS);
  MultiPlan P;
  const pw_status st = plan_multi(tris, n_tris, d_masks, offsets, hists, d_codes, cfg, P);
  if (st != PW_OK || P.items.empty()) return st;
  if (P.items.size() > (size_t)PW_NOALLOC_MAX_ITEMS)
    return set_err(PW_ERR_ARG, "%zu work items: the allocation-free call takes at most %d (use larger chunks)",
                   P.items.size(), PW_NOALLOC_MAX_ITEMS);
  int dev = 0;
  PW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaMaxDevices) return set_err(PW_ERR_ARG, "device %d beyond %d", dev, kNaMaxDevices);
  NoallocState& S = noalloc_state();
  std::lock_guard<std::mutex> lock(S.mu);
  if (!S.ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_err(PW_ERR_HIP, "hipGetSymbolAddress(scratch): %s (code %d)", hipGetErrorString(e), (int)e);
    }
    S.ptr[dev] = static_cast<unsigned char*>(p);
  }
  unsigned char* const base = S.ptr[dev];
  // ticket counter and overflow count start at zero in every call (a fill
  // kernel, not a memset: the stream may belong to a caller that records
  // graphs elsewhere)
  hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, stream, reinterpret_cast<uint64_t*>(base + kNaTicket), 2);
  PW_HIP(hipGetLastError());
  unsigned long long issued = 0;
  MultiBuffers B{reinterpret_cast<TriDesc*>(base + kNaTris),
                 reinterpret_cast<Item*>(base + kNaItems),
                 reinterpret_cast<unsigned long long*>(base + kNaTicket),
                 &issued,
                 reinterpret_cast<uint64_t*>(base + kNaOver),
                 reinterpret_cast<unsigned long long*>(base + kNaOverN),
                 (unsigned long long)PW_NOALLOC_MAX_OVERFLOW};
  return run_multi(P, B, d_masks, d_codes, stream);
}
