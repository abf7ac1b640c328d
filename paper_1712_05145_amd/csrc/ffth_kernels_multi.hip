// Multi-size launches of the FP32 inner iteration (forward y, z with the
// Green operator, inverse y, fused three-term CG x-pass): the kernels in
// ffth_kernels.h take each load's grid from its descriptor.
#include "ffth_kernels.h"
#include "ffth_launch.h"

namespace ffth {

bool multi_grid(const int n[3]) { return multi_size(n[0]) && multi_size(n[1]) && multi_size(n[2]); }

void multi_blocks(const int n[3], int out[3]) {
  out[0] = multi_y_blocks(n[0], n[1], n[2]);
  out[1] = multi_z_blocks(n[0], n[1], n[2]);
  out[2] = multi_x_blocks(n[0], n[1], n[2]);
}

hipError_t multi_ypass(const MultiSegs& sg, hipStream_t s, const Desc* d, int dir, bool h16) {
  const dim3 grid(sg.off[sg.n]);
  if (h16) hipLaunchKernelGGL(k_ypass_multi<H2>, grid, dim3(MULTI_NT), 0, s, d, dir, sg);
  else hipLaunchKernelGGL(k_ypass_multi<C2<float>>, grid, dim3(MULTI_NT), 0, s, d, dir, sg);
  return hipGetLastError();
}

hipError_t multi_zpass(const MultiSegs& sg, hipStream_t s, const Desc* d, int op, bool h16) {
  const dim3 grid(sg.off[sg.n]);
  if (h16) hipLaunchKernelGGL(k_zpass_multi<H2>, grid, dim3(MULTI_NT), 0, s, d, op, sg);
  else hipLaunchKernelGGL(k_zpass_multi<C2<float>>, grid, dim3(MULTI_NT), 0, s, d, op, sg);
  return hipGetLastError();
}

hipError_t multi_xcg3(const MultiSegs& sg, hipStream_t s, const Desc* d, bool iso, bool h16) {
  const dim3 grid(sg.off[sg.n]);
  if (iso) {
    if (h16) hipLaunchKernelGGL((k_xcg3_multi<true, H2>), grid, dim3(MULTI_NT), 0, s, d, sg);
    else hipLaunchKernelGGL((k_xcg3_multi<true, C2<float>>), grid, dim3(MULTI_NT), 0, s, d, sg);
  } else {
    if (h16) hipLaunchKernelGGL((k_xcg3_multi<false, H2>), grid, dim3(MULTI_NT), 0, s, d, sg);
    else hipLaunchKernelGGL((k_xcg3_multi<false, C2<float>>), grid, dim3(MULTI_NT), 0, s, d, sg);
  }
  return hipGetLastError();
}

}  // namespace ffth
