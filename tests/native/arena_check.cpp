// Host-only checks of the request server's arena free list: first fit,
// merging, and refusal of releases that were never handed out.
#include <cstdio>
#include <cstdlib>

#include "arena.h"

#define CHECK(c)                                               \
  do {                                                         \
    if (!(c)) {                                                \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);         \
      return 1;                                                \
    }                                                          \
  } while (0)

int main() {
  ffth::FreeList f;
  const size_t base = 4096, total = 1000;
  f.reset(base, total);
  size_t a, b, c;
  CHECK(f.alloc(300, &a) && a == base);
  CHECK(f.alloc(300, &b) && b == base + 300);
  CHECK(!f.alloc(500, &c));                       // 400 left
  // ranges that overlap free space were never handed out: refused
  CHECK(!f.release(base + 700, 50));             // inside the free tail
  CHECK(!f.release(base + 650, 100));            // straddles the free tail start
  CHECK(f.release(a, 300));                       // back: [base, base+300) free
  CHECK(!f.release(a, 300));                      // twice: refused
  CHECK(!f.release(a + 100, 10));                 // inside a free range: refused
  CHECK(f.alloc(300, &c) && c == base);           // first fit reuses the hole
  CHECK(f.release(b, 300));
  CHECK(f.release(c, 300));                       // merges with [b) and the tail
  CHECK(f.ranges().size() == 1 && f.ranges().begin()->first == base &&
        f.ranges().begin()->second == total);
  // many small allocations released out of order merge back to one range
  size_t off[10];
  for (int i = 0; i < 10; ++i) CHECK(f.alloc(100, &off[i]) && off[i] == base + 100 * (size_t)i);
  const int order[10] = {3, 7, 0, 9, 1, 5, 8, 2, 6, 4};
  for (int k = 0; k < 10; ++k) CHECK(f.release(off[order[k]], 100));
  CHECK(f.ranges().size() == 1 && f.ranges().begin()->second == total);
  CHECK(!f.release(base, 0));
  std::printf("arena free list OK\n");
  return 0;
}
