// Randomised check of the host-side arena allocator (paper_1604_07515_amd/
// csrc/arena.h) against a plain model: blocks are 256-byte aligned, never
// overlap, free + used bytes always equal the capacity, first fit returns the
// lowest-addressed free block that is large enough, and releasing everything
// coalesces the arena back into one block.  Built and run by test_arena.py.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../paper_1604_07515_amd/csrc/arena.h"

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                      \
    }                                                                \
  } while (0)

int main() {
  plc::Arena A;
  char* base = reinterpret_cast<char*>(uintptr_t(1) << 40);  // never dereferenced
  const size_t cap = size_t(1) << 24;
  A.reset(base, cap + 100);  // the odd tail is dropped
  CHECK(A.capacity() == cap && A.free_bytes() == cap && A.largest_free() == cap);
  std::mt19937_64 rng(7);
  std::map<size_t, size_t> live;  // offset -> rounded length
  size_t used = 0;
  for (int it = 0; it < 200000; it++) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      size_t want = rng() % 4 == 0 ? rng() % 65536 : rng() % 2048;
      void* p = A.alloc(want);
      size_t len = ((want ? want : 256) + 255) & ~size_t(255);
      // model: lowest gap between live blocks (or the arena ends) that fits
      size_t expect = SIZE_MAX, prev_end = 0;
      for (auto& kv : live) {
        if (kv.first - prev_end >= len) { expect = prev_end; break; }
        prev_end = kv.first + kv.second;
      }
      if (expect == SIZE_MAX && cap - prev_end >= len) expect = prev_end;
      if (expect == SIZE_MAX) {
        CHECK(p == nullptr);
        continue;
      }
      CHECK(p != nullptr);
      const size_t off = static_cast<size_t>(static_cast<char*>(p) - base);
      CHECK(off == expect && off % 256 == 0);
      live[off] = len;
      used += len;
    } else {
      auto it2 = live.begin();
      std::advance(it2, rng() % live.size());
      CHECK(A.release(base + it2->first));
      used -= it2->second;
      live.erase(it2);
    }
    CHECK(A.free_bytes() + used == cap);
  }
  CHECK(!A.release(base + 1));  // not a block start
  for (auto& kv : live) CHECK(A.release(base + kv.first));
  CHECK(A.free_bytes() == cap && A.largest_free() == cap);
  CHECK(A.release(nullptr));
  std::printf("arena ok\n");
  return 0;
}
