// scheme.hip -- single-triangulation kernels and their C-ABI entry points:
// codes of a mask batch, histogram of a mask batch, histogram of an
// enumerated index range.  One sign mask per lane (the evaluation itself is
// Eval<D>::run in pw_device.h), or for degrees 10..12 a group of four lanes
// per mask (GroupEval in pw_group.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "patchwork.h"
#include "pw_device.h"
#include "pw_group.h"
#include "pw_host.h"

namespace pw {

// ---------------------------------------------------------------- kernels
// The generic kernels walk the triangulation program in device memory; the
// bodies are shared with the kernels generated for one triangulation.

template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Cfg<D>::WAVES_PER_EU))) void k_codes(const uint32_t* __restrict__ prog, const void* __restrict__ masks,
                                               int64_t n, uint64_t* __restrict__ codes,
                                               uint32_t* __restrict__ errflag) {
  extern __shared__ uint32_t smem[];
  codes_body<D>(RtEval<D>{prog}, masks, n, codes, errflag, smem);
}

template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Cfg<D>::WAVES_PER_EU))) void k_hist(const uint32_t* __restrict__ prog, const void* __restrict__ masks,
                                              int64_t n, uint64_t index_base, const HistDev* __restrict__ h,
                                              uint64_t* __restrict__ codes, uint32_t* __restrict__ errflag) {
  extern __shared__ uint32_t smem[];
  hist_body<D>(RtEval<D>{prog}, masks, n, index_base, h, codes, errflag, smem);
}

template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Cfg<D>::WAVES_PER_EU))) void k_enum(const uint32_t* __restrict__ prog, uint64_t first, uint64_t count,
                                              Runs runs, const HistDev* __restrict__ h, uint32_t* __restrict__ errflag) {
  extern __shared__ uint32_t smem[];
  enum_body<D>(RtEval<D>{prog}, first, count, runs, h, errflag, smem);
}

// Degrees 10..12 have no kernels specialised to one triangulation, and one
// lane per mask holds a u16 entry row of up to 313 vertices plus the full
// phase-4 tables: 2-3 waves per CU.  There the kernels for one
// triangulation take a group of four lanes per mask (pw_group.h, one
// reflected quadrant per lane, full tables): 10-15 waves per CU.
constexpr int kSingleGroup = 4;
constexpr int kSingleGroupWaves = 2;  // waves per block

template <int D>
__global__ __launch_bounds__(64 * kSingleGroupWaves) void k_codes_g(const uint32_t* __restrict__ gprog,
                                                                    const void* __restrict__ masks, int64_t n,
                                                                    uint64_t* __restrict__ codes,
                                                                    uint32_t* __restrict__ errflag) {
  extern __shared__ uint32_t smem[];
  using GE = GroupEval<D, kSingleGroup>;
  using Mask = typename GE::Mask;
  constexpr int NG = GE::GC::NG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const typename GE::Mem M = GE::memory(smem + wave * GE::GC::WAVE_DW, lane);
  const int q = lane % kSingleGroup, g = lane / kSingleGroup;
  const Mask fl = GE::flip(q);
  uint32_t errs = 0;
  const int64_t waves_total = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * NG; base < n; base += waves_total * NG) {
    const int64_t i = base + g;
    const bool valid = i < n;
    const Mask m = valid ? load_mask<D>(masks, i) : (Mask)0;
    const u128 code = GE::run(const_prog(gprog), m ^ fl, M, lane, q, errs);
    if (valid && q == 0) store_code(codes, i, code);
  }
  if (errs) atomicOr(errflag, errs);
}

template <int D>
__global__ __launch_bounds__(64 * kSingleGroupWaves) void k_hist_g(const uint32_t* __restrict__ gprog,
                                                                   const void* __restrict__ masks, int64_t n,
                                                                   uint64_t index_base, const HistDev* __restrict__ h,
                                                                   uint64_t* __restrict__ codes,
                                                                   uint32_t* __restrict__ errflag) {
  extern __shared__ uint32_t smem[];
  using GE = GroupEval<D, kSingleGroup>;
  using Mask = typename GE::Mask;
  constexpr int NG = GE::GC::NG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const typename GE::Mem M = GE::memory(smem + wave * GE::GC::WAVE_DW, lane);
  const int q = lane % kSingleGroup, g = lane / kSingleGroup;
  const Mask fl = GE::flip(q);
  WaveTable tab;
  tab.clear();
  uint32_t errs = 0;
  const int64_t waves_total = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * NG; base < n; base += waves_total * NG) {
    const int64_t i = base + g;
    const bool valid = i < n && q == 0;
    const Mask m = i < n ? load_mask<D>(masks, i) : (Mask)0;
    const u128 code = GE::run(const_prog(gprog), m ^ fl, M, lane, q, errs);
    if (codes && valid) store_code(codes, i, code);
    // (the counted lanes hold increasing indices: the lowest lane of a
    // match has the smallest witness)
    tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, index_base + (uint64_t)i, lane, h);
  }
  tab.flush(h);
  if (errs) atomicOr(errflag, errs);
}

template <int D>
__global__ __launch_bounds__(64 * kSingleGroupWaves) void k_enum_g(const uint32_t* __restrict__ gprog, uint64_t first,
                                                                   uint64_t count, Runs runs,
                                                                   const HistDev* __restrict__ h,
                                                                   uint32_t* __restrict__ errflag) {
  extern __shared__ uint32_t smem[];
  using GE = GroupEval<D, kSingleGroup>;
  using Mask = typename GE::Mask;
  constexpr int NG = GE::GC::NG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const typename GE::Mem M = GE::memory(smem + wave * GE::GC::WAVE_DW, lane);
  const int q = lane % kSingleGroup, g = lane / kSingleGroup;
  const Mask fl = GE::flip(q);
  WaveTable tab;
  tab.clear();
  uint32_t errs = 0;
  const uint64_t waves_total = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wave) * NG; base < count;
       base += waves_total * NG) {
    const uint64_t k = base + (uint64_t)g;
    const bool valid = k < count && q == 0;
    const uint64_t idx = first + k;
    const u128 code = GE::run(const_prog(gprog), deposit<Mask>(idx, runs) ^ fl, M, lane, q, errs);
    tab.add_batch((uint64_t)code, (uint64_t)(code >> 64), valid, idx, lane, h);
  }
  tab.flush(h);
  if (errs) atomicOr(errflag, errs);
}

}  // namespace pw

// =================================================================== host

using namespace pw;

namespace pw {

thread_local char g_err[512] = "";

pw_status set_err(pw_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

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

}  // namespace pw

namespace {

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

// Let a kernel use up to 160 KiB of LDS in total: its dynamic part may then
// be 160 KiB minus the static parent table (set once per kernel).
template <int D>
hipError_t allow_lds(const void* kernel) {
  using C = Cfg<D>;
  const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024 - C::WAVES * C::PAR_ROWS * 64);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

// the group kernels of degrees 10..12: LDS per block, blocks for n units
template <int D>
size_t group_lds() {
  return (size_t)GCfg<D, kSingleGroup>::WAVE_DW * 4 * kSingleGroupWaves;
}
template <int D>
int group_blocks(int64_t units_per_block, int64_t n) {
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (160 * 1024) / (int64_t)group_lds<D>()));
  const int64_t need = (n + units_per_block - 1) / units_per_block;
  return (int)std::max<int64_t>(1, std::min(need, (int64_t)cu_count() * per_cu));
}
inline hipError_t allow_group_lds(const void* kernel) {
  const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}
constexpr int kGroupMasksPerBlock = 64 / kSingleGroup * kSingleGroupWaves;

template <int D>
pw_status launch_codes(const pw_tri* t, const void* masks, int64_t n, uint64_t* codes, hipStream_t s) {
  if constexpr (D >= 10) {
    static const hipError_t attr = allow_group_lds(reinterpret_cast<const void*>(&k_codes_g<D>));
    if (attr != hipSuccess) return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
    hipLaunchKernelGGL(k_codes_g<D>, dim3(group_blocks<D>(kGroupMasksPerBlock, n)), dim3(64 * kSingleGroupWaves),
                       group_lds<D>(), s, t->d_gprog[1], masks, n, codes, t->d_err);
    PW_HIP(hipGetLastError());
    return PW_OK;
  }
  using C = Cfg<D>;
  const int threads = 64 * C::WAVES;
  const size_t lds = (size_t)C::DYN_WORDS * 4 * 64 * C::WAVES;  // + the static parent table
  static const hipError_t attr = allow_lds<D>(reinterpret_cast<const void*>(&k_codes<D>));
  if (attr != hipSuccess) return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
  if (t->jit_codes && lds <= 64 * 1024) {  // module kernels keep the default 64 KiB limit
    const void* m_ = masks;
    uint64_t* c_ = codes;
    uint32_t* e_ = t->d_err;
    void* args[] = {&m_, &n, &c_, &e_};
    PW_HIP(hipModuleLaunchKernel(t->jit_codes, blocks_for<D>(threads, n), 1, 1, threads, 1, 1, (unsigned)lds, s, args,
                                 nullptr));
    return PW_OK;
  }
  hipLaunchKernelGGL(k_codes<D>, dim3(blocks_for<D>(threads, n)), dim3(threads), lds, s, t->d_prog, masks, n,
                     codes, t->d_err);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template <int D>
pw_status launch_hist(const pw_tri* t, const void* masks, int64_t n, uint64_t base, const pw_hist* h,
                      uint64_t* codes, hipStream_t s) {
  if constexpr (D >= 10) {
    static const hipError_t attr = allow_group_lds(reinterpret_cast<const void*>(&k_hist_g<D>));
    if (attr != hipSuccess) return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
    hipLaunchKernelGGL(k_hist_g<D>, dim3(group_blocks<D>(kGroupMasksPerBlock, n)), dim3(64 * kSingleGroupWaves),
                       group_lds<D>(), s, t->d_gprog[1], masks, n, base, h->d_dev, codes, t->d_err);
    PW_HIP(hipGetLastError());
    return PW_OK;
  }
  using C = Cfg<D>;
  const int threads = 64 * C::WAVES;
  const size_t lds = (size_t)C::DYN_WORDS * 4 * 64 * C::WAVES;  // + the static parent table
  static const hipError_t attr = allow_lds<D>(reinterpret_cast<const void*>(&k_hist<D>));
  if (attr != hipSuccess) return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
  if (t->jit_hist && lds <= 64 * 1024) {
    const void* m_ = masks;
    const HistDev* hd = h->d_dev;
    uint64_t* c_ = codes;
    uint32_t* e_ = t->d_err;
    void* args[] = {&m_, &n, &base, &hd, &c_, &e_};
    PW_HIP(hipModuleLaunchKernel(t->jit_hist, blocks_for<D>(threads, n), 1, 1, threads, 1, 1, (unsigned)lds, s, args,
                                 nullptr));
    return PW_OK;
  }
  hipLaunchKernelGGL(k_hist<D>, dim3(blocks_for<D>(threads, n)), dim3(threads), lds, s, t->d_prog, masks, n, base,
                     h->d_dev, codes, t->d_err);
  PW_HIP(hipGetLastError());
  return PW_OK;
}

template <int D>
pw_status launch_enum(const pw_tri* t, uint64_t first, uint64_t count, const Runs& runs, const pw_hist* h,
                      hipStream_t s) {
  if constexpr (D >= 10) {
    static const hipError_t attr = allow_group_lds(reinterpret_cast<const void*>(&k_enum_g<D>));
    if (attr != hipSuccess) return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
    const int64_t n = count > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)count;
    hipLaunchKernelGGL(k_enum_g<D>, dim3(group_blocks<D>(kGroupMasksPerBlock, n)), dim3(64 * kSingleGroupWaves),
                       group_lds<D>(), s, t->d_gprog[1], first, count, runs, h->d_dev, t->d_err);
    PW_HIP(hipGetLastError());
    return PW_OK;
  }
  using C = Cfg<D>;
  const int threads = 64 * C::WAVES;
  const size_t lds = (size_t)C::DYN_WORDS * 4 * 64 * C::WAVES;  // + the static parent table
  static const hipError_t attr = allow_lds<D>(reinterpret_cast<const void*>(&k_enum<D>));
  if (attr != hipSuccess) return set_err(PW_ERR_HIP, "hipFuncSetAttribute: %s (code %d)", hipGetErrorString(attr), (int)attr);
  const int64_t n = count > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)count;
  // the sweep kernel with a shared snapshot needs index bits 0..8 on mask
  // bits 1..9 (as when only sigma(0,0) is fixed)
  if (t->jit_enum_snap && lds <= 64 * 1024 && runs.n >= 1 && runs.src_of(0) == 0 && runs.dst_of(0) == 1 &&
      runs.len_of(0) >= 6 + kSnapBits) {
    Runs r_ = runs;
    const HistDev* hd = h->d_dev;
    uint32_t* e_ = t->d_err;
    void* args[] = {&first, &count, &r_, &hd, &e_};
    const uint64_t cs = 64ull << kSnapBits;
    const int64_t chunks = (int64_t)((first + count - 1) / cs - first / cs + 1);
    PW_HIP(hipModuleLaunchKernel(t->jit_enum_snap, blocks_for<D>(C::WAVES, chunks), 1, 1, threads, 1, 1,
                                 (unsigned)lds, s, args, nullptr));
    return PW_OK;
  }
  if (t->jit_enum && lds <= 64 * 1024) {
    Runs r_ = runs;
    const HistDev* hd = h->d_dev;
    uint32_t* e_ = t->d_err;
    void* args[] = {&first, &count, &r_, &hd, &e_};
    PW_HIP(hipModuleLaunchKernel(t->jit_enum, blocks_for<D>(threads, n), 1, 1, threads, 1, 1, (unsigned)lds, s, args,
                                 nullptr));
    return PW_OK;
  }
  hipLaunchKernelGGL(k_enum<D>, dim3(blocks_for<D>(threads, n)), dim3(threads), lds, s, t->d_prog, first, count,
                     runs, h->d_dev, t->d_err);
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
  if (d >= kGroupMinDegree) {
    for (int k = 0; k < 2; ++k) {
      rc = build_group_program(t->prog, k == 0 ? 2 : 4, t->gprog[k], msg, sizeof msg);
      if (rc != 0) {
        delete t;
        return set_err(rc, "%s", msg);
      }
      t->n_gprog[k] = group_program_words(d, k == 0 ? 2 : 4);
    }
  }
  hipError_t e = hipGetDevice(&t->device);
  if (e == hipSuccess) e = hipMalloc(&t->d_prog, sizeof(uint32_t) * t->prog.n_words);
  if (e == hipSuccess) e = hipMalloc(&t->d_err, sizeof(uint32_t));
  if (e == hipSuccess)
    e = hipMemcpy(t->d_prog, t->prog.words, sizeof(uint32_t) * t->prog.n_words, hipMemcpyHostToDevice);
  for (int k = 0; k < 2; ++k) {
    if (t->n_gprog[k] == 0) continue;
    if (e == hipSuccess) e = hipMalloc(&t->d_gprog[k], sizeof(uint32_t) * t->n_gprog[k]);
    if (e == hipSuccess)
      e = hipMemcpy(t->d_gprog[k], t->gprog[k], sizeof(uint32_t) * t->n_gprog[k], hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(t->d_err, 0, sizeof(uint32_t));
  if (e != hipSuccess) {
    if (t->d_prog) (void)hipFree(t->d_prog);
    if (t->d_err) (void)hipFree(t->d_err);
    for (uint32_t* g : t->d_gprog)
      if (g) (void)hipFree(g);
    delete t;
    return set_err(PW_ERR_HIP, "%s (code %d)", hipGetErrorString(e), (int)e);
  }
  *out = t;
  return PW_OK;
}

pw_status pw_tri_destroy(pw_tri_t t) {
  if (!t) return PW_OK;
  if (t->sweep_exec) (void)hipGraphExecDestroy(t->sweep_exec);
  if (t->cap_stream) (void)hipStreamDestroy(t->cap_stream);
  if (t->jit_mod) (void)hipModuleUnload(t->jit_mod);
  (void)hipFree(t->d_prog);
  (void)hipFree(t->d_err);
  for (uint32_t* g : t->d_gprog)
    if (g) (void)hipFree(g);
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

pw_status pw_tri_program(pw_tri_t t, uint32_t* words, int32_t cap, int32_t* n_words) {
  if (!t) return set_err(PW_ERR_ARG, "null handle");
  if (n_words) *n_words = t->prog.n_words;
  if (words) {
    if (cap < t->prog.n_words) return set_err(PW_ERR_ARG, "program has %d words, buffer %d", t->prog.n_words, cap);
    std::memcpy(words, t->prog.words, sizeof(uint32_t) * t->prog.n_words);
  }
  return PW_OK;
}

pw_status pw_tri_group_program(pw_tri_t t, int32_t G, uint32_t* words, int32_t cap, int32_t* n_words) {
  if (!t) return set_err(PW_ERR_ARG, "null handle");
  if (G != 2 && G != 4) return set_err(PW_ERR_ARG, "lane group size must be 2 or 4, got %d", G);
  const int k = G == 2 ? 0 : 1;
  if (t->n_gprog[k] == 0) return set_err(PW_ERR_ARG, "group programs exist for degrees 8..12, not %d", t->prog.d);
  if (n_words) *n_words = t->n_gprog[k];
  if (words) {
    if (cap < t->n_gprog[k]) return set_err(PW_ERR_ARG, "group program has %d words, buffer %d", t->n_gprog[k], cap);
    std::memcpy(words, t->gprog[k], sizeof(uint32_t) * t->n_gprog[k]);
  }
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
  if ((uintptr_t)codes & 15) return set_err(PW_ERR_ARG, "d_codes must be 16-byte aligned");
  PW_DISPATCH(t->prog.d, launch_codes, t, masks, n, codes, s);
}

pw_status pw_hist_create(int32_t capacity, pw_hist_t* out) {
  if (!out) return set_err(PW_ERR_ARG, "null output handle");
  *out = nullptr;
  if (capacity < 16 || capacity > (1 << 26) || (capacity & (capacity - 1)))
    return set_err(PW_ERR_ARG, "histogram capacity must be a power of two in [16, 2^26], got %d", (int)capacity);
  pw_hist* h = new (std::nothrow) pw_hist();
  if (!h) return set_err(PW_ERR_ARG, "out of host memory");
  static std::atomic<uint64_t> next_serial{1};
  h->serial = next_serial.fetch_add(1, std::memory_order_relaxed);
  h->cap = capacity;
  hipError_t e = hipMalloc(&h->state, sizeof(uint32_t) * capacity);
  if (e == hipSuccess) e = hipMalloc(&h->key, sizeof(uint64_t) * 2 * capacity);
  if (e == hipSuccess) e = hipMalloc(&h->cnt, sizeof(uint64_t) * capacity);
  if (e == hipSuccess) e = hipMalloc(&h->wit, sizeof(uint64_t) * capacity);
  if (e == hipSuccess) e = hipMalloc(&h->overflow, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&h->d_dev, sizeof(HistDev));
  if (e == hipSuccess) {
    const HistDev hd = h->dev();
    e = hipMemcpy(h->d_dev, &hd, sizeof hd, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(h->state, 0, sizeof(uint32_t) * capacity);
  if (e == hipSuccess) e = hipMemset(h->overflow, 0, sizeof(uint32_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(h->state);
    (void)hipFree(h->key);
    (void)hipFree(h->cnt);
    (void)hipFree(h->wit);
    (void)hipFree(h->overflow);
    (void)hipFree(h->d_dev);
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
  (void)hipFree(h->d_dev);
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
  PW_DISPATCH(t->prog.d, launch_hist, t, masks, n, index_base, h, nullptr, s);
}

pw_status patchwork_scheme_codes_histogram(pw_tri_t t, const void* masks, int64_t n, uint64_t index_base,
                                           uint64_t* codes, pw_hist_t h, hipStream_t s) {
  if (!t || !h) return set_err(PW_ERR_ARG, "null handle");
  if (n < 0) return set_err(PW_ERR_ARG, "negative mask count %lld", (long long)n);
  if (n == 0) return PW_OK;
  if (!masks || !codes) return set_err(PW_ERR_ARG, "null device buffer");
  if ((uintptr_t)codes & 15) return set_err(PW_ERR_ARG, "d_codes must be 16-byte aligned");
  PW_DISPATCH(t->prog.d, launch_hist, t, masks, n, index_base, h, codes, s);
}

// The runs of free bits for an enumeration and the check of its range.
static pw_status enum_plan(const pw_tri* t, uint64_t first, uint64_t count, const uint64_t fixed_zero_bits[2], Runs& runs) {
  const int nA = t->prog.nA;
  runs = Runs{};
  int nfree = 0;
  for (int b = 0; b < nA;) {
    const bool fixed = (fixed_zero_bits[b / 64] >> (b % 64)) & 1;
    if (fixed) {
      ++b;
      continue;
    }
    int e = b;
    while (e < nA && !((fixed_zero_bits[e / 64] >> (e % 64)) & 1)) ++e;
    if (runs.n == kMaxRuns) return set_err(PW_ERR_ARG, "the free bits form more than %d runs", kMaxRuns);
    runs.set(runs.n, nfree, e - b, b);
    ++runs.n;
    nfree += e - b;
    b = e;
  }
  // only the low 64 index bits are addressable
  for (int k = 0; k < runs.n; ++k) {
    if (runs.src_of(k) >= 64) {
      runs.n = k;
      break;
    }
    if (runs.src_of(k) + runs.len_of(k) > 64) runs.set(k, runs.src_of(k), 64 - runs.src_of(k), runs.dst_of(k));
  }
  if (count == 0) return PW_OK;
  if (nfree < 64) {
    const uint64_t lim = 1ull << nfree;
    if (first >= lim || count > lim - first)
      return set_err(PW_ERR_RANGE, "range exceeds 2^(free bits) (free bits %d)", nfree);
  } else if (first + count < first) {
    return set_err(PW_ERR_RANGE, "range wraps around 2^64");
  }
  return PW_OK;
}

pw_status patchwork_scheme_enumerate_range(pw_tri_t t, uint64_t first, uint64_t count,
                                           const uint64_t fixed_zero_bits[2], pw_hist_t h, hipStream_t s) {
  if (!t || !h || !fixed_zero_bits) return set_err(PW_ERR_ARG, "null argument");
  Runs runs{};
  const pw_status st = enum_plan(t, first, count, fixed_zero_bits, runs);
  if (st != PW_OK || count == 0) return st;
  PW_DISPATCH(t->prog.d, launch_enum, t, first, count, runs, h, s);
}

pw_status patchwork_scheme_sweep_graph(pw_tri_t t, uint64_t first, uint64_t count, uint64_t chunk,
                                       const uint64_t fixed_zero_bits[2], pw_hist_t h, hipStream_t s) {
  if (!t || !h || !fixed_zero_bits) return set_err(PW_ERR_ARG, "null argument");
  if (chunk == 0) return set_err(PW_ERR_ARG, "chunk must be positive");
  if (count == 0) return PW_OK;
  const uint64_t launches = (count - 1) / chunk + 1;
  if (launches > (1u << 16)) return set_err(PW_ERR_ARG, "%llu launches (at most 65536)", (unsigned long long)launches);
  // the histogram is named by its serial number, not its address: a graph
  // captured for a destroyed handle is never launched for a new one
  const uint64_t key[6] = {first, count, chunk, fixed_zero_bits[0], fixed_zero_bits[1], h->serial};
  if (!t->sweep_exec || std::memcmp(key, t->sweep_key, sizeof key) != 0) {
    if (t->sweep_exec) {
      PW_HIP(hipGraphExecDestroy(t->sweep_exec));
      t->sweep_exec = nullptr;
    }
    if (!t->cap_stream) PW_HIP(hipStreamCreateWithFlags(&t->cap_stream, hipStreamNonBlocking));
    // the range is checked before the capture (a launch failing inside it
    // would leave no graph)
    Runs runs{};
    pw_status st = enum_plan(t, first, count, fixed_zero_bits, runs);
    if (st != PW_OK) return st;
    PW_HIP(hipStreamBeginCapture(t->cap_stream, hipStreamCaptureModeRelaxed));
    for (uint64_t a = 0; a < count && st == PW_OK; a += chunk) {
      const uint64_t n = count - a < chunk ? count - a : chunk;
      st = patchwork_scheme_enumerate_range(t, first + a, n, fixed_zero_bits, h, t->cap_stream);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(t->cap_stream, &g);
    if (st != PW_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return set_err(PW_ERR_HIP, "hipStreamEndCapture: %s (code %d)", hipGetErrorString(e), (int)e);
    const hipError_t ei = hipGraphInstantiate(&t->sweep_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      t->sweep_exec = nullptr;
      return set_err(PW_ERR_HIP, "hipGraphInstantiate: %s (code %d)", hipGetErrorString(ei), (int)ei);
    }
    std::memcpy(t->sweep_key, key, sizeof key);
  }
  PW_HIP(hipGraphLaunch(t->sweep_exec, s));
  return PW_OK;
}

}  // extern "C"
