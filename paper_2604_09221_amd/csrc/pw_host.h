// pw_host.h -- host-side definitions shared by the C-ABI translation units:
// the opaque handle structs, error reporting and device queries.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "patchwork.h"
#include "pw_device.h"
#include "pw_internal.h"

struct pw_tri {
  pw::HostProgram prog;
  uint32_t* d_prog = nullptr;
  uint32_t* d_err = nullptr;
  // group programs for 2 and 4 lanes per mask (degrees 8..12, else empty)
  uint32_t gprog[2][pw::kGroupWordsMax];
  int n_gprog[2] = {0, 0};
  uint32_t* d_gprog[2] = {nullptr, nullptr};
  int device = 0;
  // kernels specialised to this triangulation (pw_tri_specialize), or null
  hipModule_t jit_mod = nullptr;
  hipFunction_t jit_codes = nullptr, jit_hist = nullptr, jit_enum = nullptr;
  hipFunction_t jit_enum_snap = nullptr;  // sweep kernel with a shared snapshot, or null
  // the chunked sweep captured by patchwork_scheme_sweep_graph, its
  // arguments and the stream it is captured on
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t sweep_exec = nullptr;
  uint64_t sweep_key[6] = {0, 0, 0, 0, 0, 0};
};

struct pw_hist {
  int32_t cap = 0;
  // process-wide serial number, never reused: a kept sweep graph names its
  // histogram by it (a freed handle's address may come back for a new one)
  uint64_t serial = 0;
  uint32_t* state = nullptr;
  uint64_t* key = nullptr;
  uint64_t* cnt = nullptr;
  uint64_t* wit = nullptr;
  uint32_t* overflow = nullptr;
  pw::HistDev* d_dev = nullptr;  // device copy of dev(), read by the kernels
  pw::HistDev dev() const { return pw::HistDev{state, key, cnt, wit, overflow, (uint32_t)(cap - 1)}; }
};

namespace pw {

// Record a message for pw_last_error() and return `code`.
__attribute__((format(printf, 2, 3))) pw_status set_err(pw_status code, const char* fmt, ...);

// Number of compute units of the current device (256 on MI355X).
int cu_count();

// Degrees for which pw_tri_specialize builds kernels (a block's LDS stays
// within the default 64 KiB of a module launch).
constexpr int kJitMaxDegree = 9;

}  // namespace pw

#define PW_HIP(call)                                                                                     \
  do {                                                                                                   \
    hipError_t e_ = (call);                                                                              \
    if (e_ != hipSuccess) return pw::set_err(PW_ERR_HIP, "%s (code %d)", hipGetErrorString(e_), (int)e_); \
  } while (0)
