// Admission order of the request server's waiting queue (host bookkeeping,
// no device calls).
#pragma once
#include <cstddef>
#include <vector>

#include "arena.h"

namespace ffth {

struct WaitInfo {
  size_t bytes;    // arena bytes the request needs
  double work;     // device work of the request (voxels x load cases)
  int bypassed;    // admissions that passed it while it waited
};

// Index of the next waiting request to admit (q in arrival order), or -1 if
// none may start now.  The request of least work whose bytes fit the free
// arena goes first (ties: the earlier arrival), so that a small request is
// not held behind a large head that waits for memory or that would occupy
// the device for much longer.  A request passed over max_bypass times is
// served first: nothing passes it any more, and it starts as soon as its
// bytes fit; so every request starts after a bounded number of others.
inline int pick_next(const std::vector<WaitInfo>& q, const FreeList& arena, int max_bypass) {
  for (size_t i = 0; i < q.size(); ++i)
    if (q[i].bypassed >= max_bypass) return arena.fits(q[i].bytes) ? (int)i : -1;
  int best = -1;
  for (size_t i = 0; i < q.size(); ++i)
    if (arena.fits(q[i].bytes) && (best < 0 || q[i].work < q[best].work)) best = (int)i;
  return best;
}

// Book the admission of q[k]: every earlier arrival was passed over once.
inline void note_admitted(std::vector<WaitInfo>& q, int k) {
  for (int i = 0; i < k; ++i) q[i].bypassed++;
}

}  // namespace ffth
