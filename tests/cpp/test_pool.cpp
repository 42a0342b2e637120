// Host-side checks of the serving pool (no device needed).
#include <assert.h>
#include <stdio.h>

#include <random>
#include <vector>

#include "../../paper_2511_04853_amd/csrc/pool.h"

int main() {
  using rl::SlabAllocator;
  SlabAllocator p(1 << 20, 256);
  // first fit, alignment, exhaustion
  uint64_t a = p.alloc(1000), b = p.alloc(256), c = p.alloc(1);
  assert(a == 0 && b == 1024 && c == 1280);
  assert(p.in_use() == 1024 + 256 + 256);
  assert(p.alloc(1 << 20) == UINT64_MAX);
  // frees coalesce back into one block
  p.release(b);
  p.release(a);
  p.release(c);
  assert(p.in_use() == 0 && p.free_blocks() == 1);
  assert(p.alloc(1 << 20) == 0);
  p.release(0);
  // fits() answers without allocating, and agrees with alloc()
  std::mt19937_64 rng(7);
  std::vector<uint64_t> live;
  for (int it = 0; it < 20000; ++it) {
    if (!live.empty() && (rng() % 3 == 0)) {
      size_t k = rng() % live.size();
      p.release(live[k]);
      live.erase(live.begin() + k);
    } else {
      std::vector<uint64_t> sz{1 + rng() % 40000, 1 + rng() % 4000};
      const bool f = p.fits(sz);
      const uint64_t before = p.in_use();
      uint64_t x = p.alloc(sz[0]);
      uint64_t y = x == UINT64_MAX ? UINT64_MAX : p.alloc(sz[1]);
      if (f) assert(x != UINT64_MAX && y != UINT64_MAX);
      if (x != UINT64_MAX) live.push_back(x);
      if (y != UINT64_MAX) live.push_back(y);
      assert(p.in_use() >= before);
    }
    assert(p.in_use() <= p.capacity());
  }
  for (auto x : live) p.release(x);
  assert(p.in_use() == 0 && p.free_blocks() == 1);
  // nearest-rank percentiles
  std::vector<double> v;
  for (int i = 1; i <= 100; ++i) v.push_back(i);
  assert(rl::percentile(v, 50) == 50 && rl::percentile(v, 99) == 99 && rl::percentile(v, 100) == 100);
  assert(rl::percentile({3.0}, 99) == 3.0);
  printf("pool ok\n");
  return 0;
}
