// Error state, launch checks and optional per-launch kernel timing of the phiks
// runtime.  Included once, by phiks.hip.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gemm_f64.hpp"
#include "phiks.h"

namespace {

using phiks::GemmArgs;

thread_local std::string g_last_error;

void set_error(const std::string& s) { g_last_error = s; }

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                   \
      return PHIKS_EDEVICE;                                                           \
    }                                                                                 \
  } while (0)

#define CHECK_LAUNCH()                                                                \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string("kernel launch: ") + hipGetErrorString(e_));              \
      return PHIKS_EDEVICE;                                                           \
    }                                                                                 \
  } while (0)

#define RET_IF(st)                                                                    \
  do {                                                                                \
    int r_ = (st);                                                                    \
    if (r_ != PHIKS_OK) return r_;                                                    \
  } while (0)

// --------------------------------------------------- kernel timing (optional)
// When enabled, every mu-mode GEMM launch carries two HIP events that record its start
// and end on its own stream, with its algorithmic flop count 2 M N K (per batch entry).
// The events ride in the kernel's own dispatch (hipExtLaunchKernelGGL), so timing adds
// no marker packets, and no idle time, between consecutive kernels.
struct TimedLaunch {
  hipEvent_t a, b;
  double flops;
  hipStream_t st;
};
std::mutex g_timing_mu;
bool g_timing = false;
std::vector<TimedLaunch> g_timed;
std::vector<hipEvent_t> g_event_pool;

bool kernel_timing_on() {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  return g_timing;
}

hipEvent_t pooled_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}


// kern<<<grid, 256>>>(args...) on st, timed as above while timing is enabled.
template <typename... KArgs, typename... Args>
int timed_launch(void (*kern)(KArgs...), unsigned grid, hipStream_t st, double flops,
                 Args... args) {
  hipEvent_t ea = nullptr, eb = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (g_timing) {
      ea = pooled_event();
      eb = pooled_event();
      if (!ea || !eb) {
        if (ea) g_event_pool.push_back(ea);
        if (eb) g_event_pool.push_back(eb);
        ea = eb = nullptr;
      }
    }
  }
  (void)hipGetLastError();  // clear a stale error left by an unrelated earlier call
  if (ea)
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, ea, eb, 0, args...);
  else
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, args...);
  CHECK_LAUNCH();
  if (ea) {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timed.push_back({ea, eb, flops, st});
  }
  return PHIKS_OK;
}

GemmArgs empty_args() {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.nb0 = g.nb1 = 1;
  return g;
}

}  // namespace
