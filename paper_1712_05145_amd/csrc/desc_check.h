// Host-side checks of launch descriptors before they are queued (plain C++,
// no device calls).
#pragma once
#include "ffth_types.h"

namespace ffth {

// A launch of the binary16-spectrum kernels reads the Green operator's FP32
// output through spec2, which only the descriptors of a binary16 inner solve
// carry; a launch of the FP32-spectrum kernels must not receive such a
// descriptor (it would read its spectrum in the wrong format).  True when all
// n descriptors match the launch's spectrum precision.
inline bool h16_launch_ok(const Desc* d, int n, bool h16) {
  for (int i = 0; i < n; ++i) {
    if (h16 ? (!d[i].h16 || d[i].spec == nullptr || d[i].spec2 == nullptr) : d[i].h16 != 0) return false;
  }
  return true;
}

}  // namespace ffth
