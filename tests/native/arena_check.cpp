// Randomised check of the device-arena bookkeeping (host only): blocks never
// overlap, stay inside the arena and aligned, releases coalesce so that after
// everything is released the arena is one free block again, and top-end
// allocations leave the bottom contiguous.
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <random>
#include <vector>

#include "../../paper_1703_02438_amd/csrc/arena.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main() {
  using nk::Arena;
  const uint64_t cap = 1 << 20;
  const uint64_t pages = cap / Arena::kAlign;
  for (int seed = 0; seed < 20; ++seed) {
    std::mt19937_64 rng(seed);
    Arena a(cap);
    std::vector<int> owner(pages, -1);  // page -> block id (model)
    std::map<uint64_t, std::pair<uint64_t, int>> live;  // off -> (len, id)
    int next_id = 0;
    for (int step = 0; step < 4000; ++step) {
      const bool do_alloc = live.empty() || (rng() % 100) < 55;
      if (do_alloc) {
        const uint64_t want = 1 + rng() % (cap / 16);
        const bool top = rng() % 4 == 0;
        const uint64_t off = top ? a.alloc_top(want) : a.alloc(want);
        // model: is there any run of free pages long enough?
        const uint64_t need = (want + Arena::kAlign - 1) / Arena::kAlign;
        uint64_t run = 0, best = 0;
        for (uint64_t p = 0; p < pages; ++p) {
          run = owner[p] < 0 ? run + 1 : 0;
          best = run > best ? run : best;
        }
        if (off == Arena::kFail) {
          CHECK(best < need);
          continue;
        }
        CHECK(off % Arena::kAlign == 0);
        CHECK(off + need * Arena::kAlign <= cap);
        const int id = next_id++;
        for (uint64_t p = off / Arena::kAlign; p < off / Arena::kAlign + need; ++p) {
          CHECK(owner[p] < 0);
          owner[p] = id;
        }
        live[off] = {need, id};
      } else {
        auto it = live.begin();
        std::advance(it, rng() % live.size());
        CHECK(a.release(it->first));
        for (uint64_t p = it->first / Arena::kAlign; p < it->first / Arena::kAlign + it->second.first;
             ++p)
          owner[p] = -1;
        live.erase(it);
      }
      uint64_t used = 0;
      for (const auto& l : live) used += l.second.first * Arena::kAlign;
      CHECK(a.in_use() == used);
      CHECK(a.used_blocks() == live.size());
      CHECK(!a.release(cap + 256));  // not a block
    }
    for (const auto& l : live) CHECK(a.release(l.first));
    CHECK(a.in_use() == 0);
    CHECK(a.free_blocks() == 1);
    CHECK(a.largest_free() == cap);
  }
  {  // long-lived blocks from the top, short-lived from the bottom
    Arena a(cap);
    const uint64_t t0 = a.alloc_top(1000), t1 = a.alloc_top(5000);
    CHECK(t0 == cap - 1024 && t1 == cap - 1024 - 5120);
    std::vector<uint64_t> tmp;
    for (int i = 0; i < 50; ++i) tmp.push_back(a.alloc(3000 + i));
    for (size_t i = 0; i < tmp.size(); i += 2) CHECK(a.release(tmp[i]));
    for (size_t i = 1; i < tmp.size(); i += 2) CHECK(a.release(tmp[i]));
    CHECK(a.free_blocks() == 1);
    CHECK(a.largest_free() == cap - 1024 - 5120);
    CHECK(a.peak() >= 1024 + 5120);
    CHECK(a.alloc(cap) == Arena::kFail);
    CHECK(Arena(100).capacity() == 0 && Arena(100).alloc(1) == Arena::kFail);
  }
  printf("arena ok\n");
  return 0;
}
