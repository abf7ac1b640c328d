// Host-only checks of the request server's admission order: least work
// first among requests that fit, bounded bypassing of a waiting request.
#include <cstdio>
#include <vector>

#include "admission.h"

#define CHECK(c)                                               \
  do {                                                         \
    if (!(c)) {                                                \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);         \
      return 1;                                                \
    }                                                          \
  } while (0)

using ffth::WaitInfo;

// Admit from q (arrival order) into arena until pick_next refuses; returns the
// admitted original indices in admission order.
static std::vector<int> drain(std::vector<WaitInfo> q, ffth::FreeList& arena, int max_bypass, int slots) {
  std::vector<int> id(q.size()), out;
  for (size_t i = 0; i < q.size(); ++i) id[i] = (int)i;
  while ((int)out.size() < slots) {
    const int k = ffth::pick_next(q, arena, max_bypass);
    if (k < 0) break;
    size_t off;
    if (!arena.alloc(q[k].bytes, &off)) return {-1};
    ffth::note_admitted(q, k);
    out.push_back(id[k]);
    q.erase(q.begin() + k);
    id.erase(id.begin() + k);
  }
  return out;
}

int main() {
  // smallest work first among those that fit; ties by arrival
  {
    ffth::FreeList a;
    a.reset(0, 1000);
    std::vector<WaitInfo> q = {{600, 8.0, 0}, {100, 1.0, 0}, {100, 1.0, 0}, {300, 2.0, 0}};
    std::vector<int> got = drain(q, a, 100, 10);
    CHECK((got == std::vector<int>{1, 2, 3}));            // 600 no longer fits after the others
  }
  // a head that does not fit does not block smaller requests behind it
  {
    ffth::FreeList a;
    a.reset(0, 500);
    std::vector<WaitInfo> q = {{800, 9.0, 0}, {200, 1.0, 0}, {200, 3.0, 0}};
    std::vector<int> got = drain(q, a, 100, 10);
    CHECK((got == std::vector<int>{1, 2}));
  }
  // a request passed over max_bypass times goes first and blocks the rest
  {
    ffth::FreeList a;
    a.reset(0, 1000);
    std::vector<WaitInfo> q = {{700, 9.0, 2}, {100, 1.0, 0}};
    CHECK(ffth::pick_next(q, a, 2) == 0);
    size_t off;
    CHECK(a.alloc(400, &off));                            // 600 left: the starved head does not fit
    CHECK(ffth::pick_next(q, a, 2) == -1);                // and nothing passes it
    CHECK(ffth::pick_next(q, a, 3) == 1);                 // with a larger bound the small one goes
  }
  // bypass counts grow only for earlier arrivals
  {
    std::vector<WaitInfo> q = {{1, 5.0, 0}, {1, 4.0, 0}, {1, 1.0, 0}, {1, 7.0, 0}};
    ffth::note_admitted(q, 2);
    CHECK(q[0].bypassed == 1 && q[1].bypassed == 1 && q[2].bypassed == 0 && q[3].bypassed == 0);
  }
  // bounded wait: with a stream of small arrivals a large request is admitted
  // after at most max_bypass others
  {
    ffth::FreeList a;
    a.reset(0, 1000);
    std::vector<WaitInfo> q = {{900, 50.0, 0}};
    const int B = 3;
    int admitted_small = 0;
    bool big_in = false;
    std::vector<size_t> offs;
    for (int t = 0; t < 20 && !big_in; ++t) {
      q.push_back({100, 1.0, 0});                         // a small request arrives
      const int k = ffth::pick_next(q, a, B);
      if (k < 0) {                                        // free everything: the running ones finish
        a.reset(0, 1000);
        continue;
      }
      size_t off;
      CHECK(a.alloc(q[k].bytes, &off));
      ffth::note_admitted(q, k);
      if (q[k].work == 50.0) big_in = true;
      else admitted_small++;
      q.erase(q.begin() + k);
    }
    CHECK(big_in && admitted_small <= B);
  }
  std::printf("admission order OK\n");
  return 0;
}
