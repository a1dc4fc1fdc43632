// Error state, launch checks and optional per-launch kernel timing of the phiks
// runtime.  Included once, by phiks.hip.
#pragma once
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
// When enabled, every mu-mode GEMM launch is bracketed by two HIP events recorded
// on its own stream, with its algorithmic flop count 2 M N K (per batch entry).
struct TimedLaunch {
  hipEvent_t a, b;
  double flops;
};
std::mutex g_timing_mu;
bool g_timing = false;
std::vector<TimedLaunch> g_timed;
std::vector<hipEvent_t> g_event_pool;

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


GemmArgs empty_args() {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.nb0 = g.nb1 = 1;
  return g;
}

}  // namespace
