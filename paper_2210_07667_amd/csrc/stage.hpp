// Pinned staging of the small host-to-device tables that a plan build uploads (shifted
// operators, pointer arrays of the batched GEMMs, Taylor and scale jobs).  A copy from
// pageable host memory makes the runtime wait for the stream, so a plan built while an
// earlier phi-action is still queued would stall the host until that work drains and
// leave the device idle while the host plans.  Sources staged in pinned memory make
// every upload a truly asynchronous copy.
//
// Host side: a per-device pool of pinned blocks.  A build fills one block at a time;
// a filled block is retired with an event recorded on the build's stream after its
// last copy, and is reused only once that event has completed.  At most kMaxBlocks
// blocks stay pinned per device; past that the host waits for the oldest one.
// Device side: tables are carved from chunks allocated in stream order and freed in
// stream order when the build ends, after every kernel that reads them was enqueued.
// Deferred mode: each separate upload costs a copy launch of its own on the stream, so
// a build may hold its uploads and record its launches, then submit them: the uploads
// go out as one copy per contiguous run, followed by the launches in recorded order.
// Included once, by phiks.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <vector>

#include "runtime.hpp"
#include "stage_runs.hpp"

namespace {

struct StageBlock {
  char* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;   // recorded after the block's last copy
};

class StagePool {
 public:
  static constexpr size_t kBlockBytes = size_t(4) << 20;
  static constexpr size_t kMaxBlocks = 16;

  // A block of at least `need` bytes whose earlier copies have all completed.
  int acquire(int device, size_t need, StageBlock& out) {
    std::unique_lock<std::mutex> lk(mu_);
    Dev& D = dev(device);
    for (;;) {
      // pending blocks whose copies are done become idle (oldest first)
      while (!D.pending.empty() && hipEventQuery(D.pending.front().done) == hipSuccess) {
        D.idle.push_back(D.pending.front());
        D.pending.pop_front();
      }
      int best = -1;
      for (size_t i = 0; i < D.idle.size(); ++i)
        if (D.idle[i].cap >= need && (best < 0 || D.idle[i].cap < D.idle[(size_t)best].cap)) best = (int)i;
      if (best >= 0) {
        out = D.idle[(size_t)best];
        D.idle.erase(D.idle.begin() + best);
        return PHIKS_OK;
      }
      if (D.idle.size() + D.pending.size() + D.out < kMaxBlocks || D.pending.empty()) break;
      // every block is in flight: wait for the oldest
      hipEvent_t e = D.pending.front().done;
      lk.unlock();
      (void)hipEventSynchronize(e);
      lk.lock();
    }
    // a new block (an idle one too small for `need` is replaced)
    if (!D.idle.empty() && D.idle.size() + D.pending.size() + D.out >= kMaxBlocks) {
      StageBlock old = D.idle.back();
      D.idle.pop_back();
      (void)hipHostFree(old.host);
      (void)hipEventDestroy(old.done);
    }
    StageBlock b;
    b.cap = std::max(kBlockBytes, (need + kBlockBytes - 1) / kBlockBytes * kBlockBytes);
    if (hipHostMalloc((void**)&b.host, b.cap, hipHostMallocDefault) != hipSuccess) {
      set_error("hipHostMalloc of a staging block failed");
      return PHIKS_ENOMEM;
    }
    if (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipHostFree(b.host);
      set_error("hipEventCreate for a staging block failed");
      return PHIKS_EDEVICE;
    }
    out = b;
    return PHIKS_OK;
  }

  void checked_out(int device, int delta) {
    std::lock_guard<std::mutex> lk(mu_);
    dev(device).out += delta;
  }

  // Returns a block; its copies were enqueued on `st` (the device must be current).
  void retire(int device, StageBlock b, hipStream_t st) {
    const bool recorded = hipEventRecord(b.done, st) == hipSuccess;
    if (!recorded) (void)hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lk(mu_);
    Dev& D = dev(device);
    if (recorded)
      D.pending.push_back(b);
    else
      D.idle.push_back(b);
  }

 private:
  struct Dev {
    int id = -1;
    std::vector<StageBlock> idle;
    std::deque<StageBlock> pending;
    size_t out = 0;   // blocks held by builds in progress
  };
  Dev& dev(int device) {
    for (Dev& D : devs_)
      if (D.id == device) return D;
    devs_.emplace_back();
    devs_.back().id = device;
    return devs_.back();
  }
  std::mutex mu_;
  std::deque<Dev> devs_;   // deque: references stay valid as devices are added
};

StagePool g_stage_pool;

// The uploads of one build, all on one stream.  finish() (or the destructor) retires
// the pinned block and frees the device chunks in stream order.
class Stager {
 public:
  explicit Stager(hipStream_t st) : st_(st) { (void)hipGetDevice(&device_); }
  Stager(const Stager&) = delete;
  Stager& operator=(const Stager&) = delete;
  ~Stager() { (void)finish(); }

  // Enqueues the copy of `bytes` from host `src` to device `dst`; src may be reused
  // as soon as this returns.
  int upload(void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return PHIKS_OK;
    char* h = nullptr;
    RET_IF(host_space(bytes, h));
    std::memcpy(h, src, bytes);
    if (deferred_) {
      pending_.push_back({static_cast<char*>(dst), h, bytes, chunk_of(dst, bytes)});
      return PHIKS_OK;
    }
    HIP_OK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, st_));
    return PHIKS_OK;
  }

  // Device memory of `bytes` for the kernels enqueued before finish(), which frees it
  // (stream-ordered).
  int scratch(size_t bytes, void** d) {
    *d = nullptr;
    return device_space(bytes, reinterpret_cast<char**>(d));
  }

  // Holds uploads and records launches from here on, until submit().
  void defer() { deferred_ = true; }

  // Runs `f` (a launch or another stream-ordered call) now, or at submit() when deferred.
  int later(std::function<int()> f) {
    if (!deferred_) return f();
    launches_.push_back(std::move(f));
    return PHIKS_OK;
  }

  // Issues the held uploads, then the recorded launches in order; leaves deferred mode.
  int submit() {
    RET_IF(issue_copies());
    deferred_ = false;
    std::vector<std::function<int()>> fs;
    fs.swap(launches_);
    for (auto& f : fs) RET_IF(f());
    return PHIKS_OK;
  }

  // A device copy of a host table, valid for the kernels enqueued on the stream
  // before finish().
  template <typename T>
  int table(const T* src, size_t count, T** dev) {
    const size_t bytes = count * sizeof(T);
    *dev = nullptr;
    RET_IF(device_space(bytes, reinterpret_cast<char**>(dev)));
    return upload(*dev, src, bytes);
  }

  int finish() {
    int rc = PHIKS_OK;
    // a build that failed before submit(): nothing recorded reaches the stream
    launches_.clear();
    pending_.clear();
    deferred_ = false;
    if (have_) {
      g_stage_pool.retire(device_, blk_, st_);
      g_stage_pool.checked_out(device_, -1);
      have_ = false;
    }
    for (char* c : chunks_)
      if (hipFreeAsync(c, st_) != hipSuccess) rc = PHIKS_EDEVICE;
    chunks_.clear();
    chunk_caps_.clear();
    chunk_used_ = chunk_cap_ = 0;
    return rc;
  }

 private:
  static size_t align(size_t x) { return phiks::staged_align(x); }

  // Index of the device chunk that holds [dst, dst + bytes), or -1.
  int chunk_of(const void* dst, size_t bytes) const {
    const char* d = static_cast<const char*>(dst);
    for (size_t c = 0; c < chunks_.size(); ++c)
      if (d >= chunks_[c] && d + bytes <= chunks_[c] + chunk_caps_[c]) return (int)c;
    return -1;
  }

  // One copy per run of held uploads that follow each other in the pinned block and in
  // one device chunk alike (phiks::staged_run_end; the padding in between belongs to the
  // same block and chunk).
  int issue_copies() {
    size_t i = 0;
    while (i < pending_.size()) {
      const size_t j = phiks::staged_run_end(pending_.data(), pending_.size(), i);
      const size_t bytes = (size_t)(pending_[j - 1].dst - pending_[i].dst) + pending_[j - 1].bytes;
      HIP_OK(hipMemcpyAsync(pending_[i].dst, pending_[i].host, bytes, hipMemcpyHostToDevice, st_));
      i = j;
    }
    pending_.clear();
    return PHIKS_OK;
  }

  int host_space(size_t bytes, char*& h) {
    if (!have_ || used_ + bytes > blk_.cap) {
      if (have_) {
        RET_IF(issue_copies());   // the block's held uploads go out before it is retired
        g_stage_pool.retire(device_, blk_, st_);
        g_stage_pool.checked_out(device_, -1);
        have_ = false;
      }
      RET_IF(g_stage_pool.acquire(device_, bytes, blk_));
      g_stage_pool.checked_out(device_, 1);
      have_ = true;
      used_ = 0;
    }
    h = blk_.host + used_;
    used_ = align(used_ + bytes);
    return PHIKS_OK;
  }

  int device_space(size_t bytes, char** d) {
    if (chunks_.empty() || chunk_used_ + bytes > chunk_cap_) {
      const size_t cap = std::max(kChunkBytes, align(bytes));
      char* c = nullptr;
      HIP_OK(hipMallocAsync((void**)&c, cap, st_));
      chunks_.push_back(c);
      chunk_caps_.push_back(cap);
      chunk_used_ = 0;
      chunk_cap_ = cap;
    }
    *d = chunks_.back() + chunk_used_;
    chunk_used_ = align(chunk_used_ + bytes);
    return PHIKS_OK;
  }

  static constexpr size_t kChunkBytes = size_t(1) << 20;
  hipStream_t st_;
  int device_ = 0;
  StageBlock blk_;
  bool have_ = false;
  size_t used_ = 0;
  std::vector<char*> chunks_;
  std::vector<size_t> chunk_caps_;
  size_t chunk_used_ = 0, chunk_cap_ = 0;
  bool deferred_ = false;
  std::vector<phiks::StagedCopy> pending_;
  std::vector<std::function<int()>> launches_;
};

}  // namespace
