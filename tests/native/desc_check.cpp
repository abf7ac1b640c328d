// Host-only checks of the descriptor test that guards binary16 launches.
#include <cstdio>
#include <cstring>
#include <vector>

#include "desc_check.h"

#define CHECK(c)                                               \
  do {                                                         \
    if (!(c)) {                                                \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);         \
      return 1;                                                \
    }                                                          \
  } while (0)

int main() {
  using ffth::Desc;
  static float spec_buf[64], copy_buf[64];
  std::vector<Desc> d(3);
  for (auto& x : d) {
    std::memset(&x, 0, sizeof(Desc));
    x.spec = spec_buf;
  }
  // FP32 spectrum: plain descriptors pass, empty launches pass
  CHECK(ffth::h16_launch_ok(d.data(), 3, false));
  CHECK(ffth::h16_launch_ok(d.data(), 0, true));
  // binary16 launch of FP32 descriptors: refused (spec2 would be null)
  CHECK(!ffth::h16_launch_ok(d.data(), 3, true));
  for (auto& x : d) {
    x.h16 = 1;
    x.spec2 = copy_buf;
  }
  CHECK(ffth::h16_launch_ok(d.data(), 3, true));
  // binary16 descriptors in an FP32-spectrum launch: refused
  CHECK(!ffth::h16_launch_ok(d.data(), 3, false));
  // one descriptor without its FP32 copy among binary16 ones: refused
  d[1].spec2 = nullptr;
  CHECK(!ffth::h16_launch_ok(d.data(), 3, true));
  CHECK(ffth::h16_launch_ok(d.data(), 1, true));      // only the first one launched
  // flag set without the copy buffer (a descriptor built for another plan)
  d[1].spec2 = copy_buf;
  d[2].h16 = 0;
  CHECK(!ffth::h16_launch_ok(d.data(), 3, true));
  std::printf("descriptor checks OK\n");
  return 0;
}
