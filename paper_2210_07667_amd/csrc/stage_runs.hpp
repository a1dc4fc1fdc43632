// Which held host-to-device uploads of a staging ring may go out as one copy (the
// deferred mode of Stager, stage.hpp).  No HIP dependency, so that host tests can
// include it alone.
#pragma once
#include <cstddef>

namespace phiks {

// One held upload: `bytes` from the pinned block at `host` to device `dst`.  `chunk` is
// the index of the device allocation (a chunk of the stager) that holds the whole
// destination, or -1 when the destination lies in memory the stager did not allocate.
struct StagedCopy {
  char* dst;
  const char* host;
  size_t bytes;
  int chunk;
};

inline size_t staged_align(size_t x) { return (x + 255) & ~size_t(255); }

// End (exclusive) of the run of held uploads that starts at v[i] and may be joined into
// one copy: each next entry starts where the previous one's 256-byte-rounded extent ends,
// on the device and in the pinned block alike, and lies in the same device chunk.  The
// chunk test matters: two separate allocations can be adjacent in the address space,
// and a copy must not span two allocations.
inline size_t staged_run_end(const StagedCopy* v, size_t n, size_t i) {
  size_t j = i + 1;
  while (j < n && v[j].chunk >= 0 && v[j].chunk == v[j - 1].chunk &&
         v[j].dst == v[j - 1].dst + staged_align(v[j - 1].bytes) &&
         v[j].host == v[j - 1].host + staged_align(v[j - 1].bytes))
    ++j;
  return j;
}

}  // namespace phiks
