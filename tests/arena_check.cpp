// Randomised check of the served form's request-state allocator (host-only)
// against a plain model: a byte map of the arena in 256-byte granules.
// Every allocation must lie inside the arena, overlap no live block, start
// at the lowest granule where a free run of its rounded size begins (first
// fit), and fail only when no such run exists; the byte count in use must
// follow; after everything is released, one allocation of the whole arena
// must succeed again (the free blocks coalesced).
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "arena.h"

int main() {
  const int64_t G = 256;
  int fails = 0;
  for (int trial = 0; trial < 40; trial++) {
    std::mt19937_64 rng(1000 + trial);
    const int64_t granules = 64 + (int64_t)(rng() % 512);
    const int64_t size = granules * G - (trial % 2 ? 100 : 0);  // a ragged end on odd trials
    const int64_t usable = size / G;                              // whole granules the model can hand out
    pg::Arena a;
    a.reset(size);
    std::vector<int> owner(granules, -1);
    struct Blk { int64_t off, len; };
    std::vector<Blk> live;
    int64_t used = 0;
    for (int step = 0; step < 4000; step++) {
      const bool do_alloc = live.empty() || (rng() % 100) < 55;
      if (do_alloc) {
        const int64_t len = 1 + (int64_t)(rng() % (G * 24));
        const int64_t need = (len + G - 1) / G;
        // first fit in the model
        int64_t want = -1, run = 0;
        for (int64_t g = 0; g < usable; g++) {
          run = owner[g] < 0 ? run + 1 : 0;
          if (run == need) {
            want = g - need + 1;
            break;
          }
        }
        // a run that would end in the ragged tail only fits if the tail is whole
        const int64_t off = a.alloc(len);
        if (off < 0) {
          if (want >= 0) fails++;
          continue;
        }
        if (off % G || off / G != want || off + need * G > granules * G) fails++;
        for (int64_t g = off / G; g < off / G + need && g < granules; g++) {
          if (owner[g] >= 0) fails++;
          owner[g] = (int)live.size();
        }
        live.push_back({off, len});
        used += need * G;
      } else {
        const size_t k = rng() % live.size();
        const Blk b = live[k];
        a.release(b.off, b.len);
        const int64_t need = (b.len + G - 1) / G;
        for (int64_t g = b.off / G; g < b.off / G + need; g++) owner[g] = -1;
        live[k] = live.back();
        live.pop_back();
        for (int64_t g = 0; g < granules; g++)
          if (owner[g] == (int)live.size()) owner[g] = (int)k;  // the moved block's index
        used -= need * G;
      }
      if (a.used.load() != used) fails++;
    }
    for (const Blk &b : live) a.release(b.off, b.len);
    if (a.used.load() != 0) fails++;
    if (a.alloc(usable * G) != 0) fails++;
  }
  std::printf("failures %d\n", fails);
  return fails == 0 ? 0 : 1;
}
