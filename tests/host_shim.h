// Host shim for tests/test_host_emulation.py and tests/test_group_emulation.py:
// lets g++ compile the device headers (pw_device.h, pw_group.h) and a
// generated per-triangulation evaluator, so the evaluation runs on the CPU.
// Wave-level intrinsics (ballots, shuffles, lane reads) and global atomics
// are not emulated and abort if reached.  atomicOr is a plain OR: the
// emulation runs one lane at a time, so nothing can interleave with it
// (the sweep kernel's per-chunk stages use it on the wave's own LDS words).
#pragma once
#define __HIPCC_RTC__ 1
#include <cstdint>
#include <cstdio>
#include <cstdlib>
namespace __hip_internal {
typedef ::uint8_t uint8_t;
typedef ::uint16_t uint16_t;
typedef ::uint32_t uint32_t;
typedef ::uint64_t uint64_t;
typedef ::int64_t int64_t;
}
#define __device__
#define __host__
#define __global__
#define __shared__
#define __restrict__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
struct Dim3E { unsigned x, y, z; };
extern Dim3E threadIdx, blockIdx, blockDim, gridDim;
static inline int __clzll(long long x) { return x ? __builtin_clzll((unsigned long long)x) : 64; }
static inline int __clz(int x) { return x ? __builtin_clz((unsigned)x) : 32; }
static inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
static inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
static inline int __popc(unsigned x) { return __builtin_popcount(x); }
[[noreturn]] static inline void emu_unsupported() { std::fprintf(stderr, "unsupported in emulation\n"); std::abort(); }
template <class T> static inline T atomicAdd(T*, T) { emu_unsupported(); }
template <class T> static inline T atomicMin(T*, T) { emu_unsupported(); }
template <class T> static inline T atomicOr(T* p, T x) {
  const T old = *p;
  *p = old | x;
  return old;
}
static inline uint64_t __ballot(int) { emu_unsupported(); }
static inline int __shfl_xor(int, int, int) { emu_unsupported(); }
static inline uint64_t __builtin_amdgcn_ballot_w64(bool) { emu_unsupported(); }
static inline int emu_readlane(int, int) { emu_unsupported(); }
#define __builtin_amdgcn_readlane(a, b) emu_readlane(a, b)
#define __builtin_amdgcn_readfirstlane(a) ((int)(a))  // returns int on the device too
#define __HIP_MEMORY_SCOPE_AGENT 0
template <class T> static inline T __hip_atomic_load(T*, int, int) { emu_unsupported(); }
template <class T> static inline void __hip_atomic_store(T*, T, int, int) { emu_unsupported(); }
template <class T> static inline bool __hip_atomic_compare_exchange_strong(T*, T*, T, int, int, int) { emu_unsupported(); }
#define PW_OPAQUE(x) asm volatile("" : "+r"(x))
#define PW_OPAQUE_S(x) asm volatile("" : "+r"(x))
#define __builtin_amdgcn_wave_barrier() ((void)0)
