// The run rule of the deferred staging uploads (csrc/stage_runs.hpp): which held
// uploads go out as one copy.  A copy must stay inside one device allocation, so runs
// never cross from one device chunk into the next, even where the chunks are adjacent in
// the address space (a chunk filled exactly by 256-byte-rounded tables, followed by a
// new chunk that the allocator placed right after it).
//   stage_runs_check      exit status 0 when every check holds
#include <cstdio>
#include <cstdint>
#include <vector>

#include "stage_runs.hpp"

using phiks::StagedCopy;
using phiks::staged_align;
using phiks::staged_run_end;

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

// A fake stager: device chunks of 1 MiB (or one table's rounded size) placed one after
// the other in a fake address space, one pinned block; tables carved and held as Stager
// does, with the chunk index Stager records.
struct FakeStager {
  std::vector<char*> base;
  std::vector<size_t> cap;
  size_t used = 0, host_used = 0;
  char* next_chunk;
  char* host;
  std::vector<StagedCopy> held;
  FakeStager(char* dev0, char* host0) : next_chunk(dev0), host(host0) {}
  void table(size_t bytes) {
    if (base.empty() || used + bytes > cap.back()) {
      const size_t c = std::max<size_t>(size_t(1) << 20, staged_align(bytes));
      base.push_back(next_chunk);
      cap.push_back(c);
      next_chunk += c;   // the next chunk starts right where this one ends
      used = 0;
    }
    char* d = base.back() + used;
    used = staged_align(used + bytes);
    held.push_back({d, host + host_used, bytes, (int)base.size() - 1});
    host_used = staged_align(host_used + bytes);
  }
};

int main() {
  char* const D = reinterpret_cast<char*>(uintptr_t(1) << 40);
  char* const H = reinterpret_cast<char*>(uintptr_t(1) << 36);
  {  // contiguous in one chunk and one block: one run
    StagedCopy v[2] = {{D, H, 100, 0}, {D + 256, H + 256, 8, 0}};
    CHECK(staged_run_end(v, 2, 0) == 2);
  }
  {  // adjacent addresses, two chunks: two runs
    StagedCopy v[2] = {{D, H, 256, 0}, {D + 256, H + 256, 8, 1}};
    CHECK(staged_run_end(v, 2, 0) == 1);
  }
  {  // destination not in a stager chunk: never joined
    StagedCopy v[2] = {{D, H, 256, -1}, {D + 256, H + 256, 8, -1}};
    CHECK(staged_run_end(v, 2, 0) == 1);
  }
  {  // the next entry starts at the unrounded end: not the stager's layout, not joined
    StagedCopy v[2] = {{D, H, 100, 0}, {D + 100, H + 100, 8, 0}};
    CHECK(staged_run_end(v, 2, 0) == 1);
  }
  {  // contiguous on the device, not in the pinned block
    StagedCopy v[2] = {{D, H, 256, 0}, {D + 256, H + 512, 8, 0}};
    CHECK(staged_run_end(v, 2, 0) == 1);
  }
  {  // many one-slot tables fill the first chunk exactly; the second chunk follows it
    FakeStager S(D, H);
    S.table(size_t(1) << 19);                      // a work buffer of half a chunk
    for (int t = 0; t < 3000; ++t) S.table(24 + 8 * (t % 4));
    CHECK(S.base.size() >= 2 && S.base[1] == S.base[0] + S.cap[0]);
    bool exact_fill = false;
    for (size_t i = 0; i + 1 < S.held.size(); ++i)
      if (S.held[i].chunk == 0 && S.held[i + 1].chunk == 1 &&
          S.held[i + 1].dst == S.held[i].dst + staged_align(S.held[i].bytes))
        exact_fill = true;
    CHECK(exact_fill);   // the case the chunk test exists for
    size_t runs = 0;
    for (size_t i = 0; i < S.held.size();) {
      const size_t j = staged_run_end(S.held.data(), S.held.size(), i);
      CHECK(j > i);
      const StagedCopy& a = S.held[i];
      const StagedCopy& b = S.held[j - 1];
      const size_t bytes = (size_t)(b.dst - a.dst) + b.bytes;
      const int c = a.chunk;
      CHECK(a.dst >= S.base[c] && a.dst + bytes <= S.base[c] + S.cap[c]);   // one allocation
      CHECK(b.host + b.bytes == a.host + bytes);                            // same extent on the host
      ++runs;
      i = j;
    }
    CHECK(runs == S.base.size());   // one copy per chunk
  }
  if (failures) return 1;
  std::printf("stage runs check passed\n");
  return 0;
}
