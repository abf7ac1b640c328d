// Instantiations of the FFT-pass kernels for one precision (FFTH_REAL is
// float or double, set on the compiler command line) and every axis length
// in FFTH_SIZES.
#include "ffth_kernels.h"
#include "ffth_launch.h"

#ifndef FFTH_REAL
#error "compile with -DFFTH_REAL=float or -DFFTH_REAL=double"
#endif

namespace ffth {

using R = FFTH_REAL;

template <typename T> int Launch<T>::x_rows(int n) {
#define FFTH_CASE(N) if (n == N) return ffth::x_rows<T>(N);
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return 0;
}
template <typename T> int Launch<T>::xi_rows(int n) {
#define FFTH_CASE(N) if (n == N) return ffth::xi_rows<T>(N);
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return 0;
}
template <typename T> int Launch<T>::y_cols(int n) {
#define FFTH_CASE(N) if (n == N) return ffth::y_cols<T>(N);
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return 0;
}
template <typename T> int Launch<T>::z_cols(int n) {
#define FFTH_CASE(N) if (n == N) return ffth::z_cols<T>(N);
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return 0;
}

template <typename T> hipError_t Launch<T>::xfwd(int n2, bool iso, dim3 grid, hipStream_t s, const Desc* d, int mode, long rows,
                                       long nvox) {
#define FFTH_CASE(N)                                                                                          \
  if (n2 == N) {                                                                                              \
    if (iso) hipLaunchKernelGGL((k_xfwd<T, N, true>), grid, dim3(NT), 0, s, d, mode, rows, nvox);  \
    else hipLaunchKernelGGL((k_xfwd<T, N, false>), grid, dim3(NT), 0, s, d, mode, rows, nvox);     \
    return hipGetLastError();                                                                                 \
  }
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template <typename T> hipError_t Launch<T>::xinv(int n2, bool iso, dim3 grid, hipStream_t s, const Desc* d, int mode, long rows,
                                       long nvox) {
#define FFTH_CASE(N)                                                                                          \
  if (n2 == N) {                                                                                              \
    if (iso) hipLaunchKernelGGL((k_xinv<T, N, true>), grid, dim3(NT), 0, s, d, mode, rows, nvox);  \
    else hipLaunchKernelGGL((k_xinv<T, N, false>), grid, dim3(NT), 0, s, d, mode, rows, nvox);     \
    return hipGetLastError();                                                                                 \
  }
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template <typename T> hipError_t Launch<T>::ypass(int n1, dim3 grid, hipStream_t s, const Desc* d, int dir, int ncols,
                                        int ntiles) {
#define FFTH_CASE(N)                                                                                  \
  if (n1 == N) {                                                                                      \
    hipLaunchKernelGGL((k_ypass<T, N>), grid, dim3(ffth::y_threads<T>(N)), 0, s, d, dir, ncols, ntiles); \
    return hipGetLastError();                                                                         \
  }
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template <typename T> hipError_t Launch<T>::zpass(int n0, dim3 grid, hipStream_t s, const Desc* d, int op, int n1, int h,
                                        double scale) {
#define FFTH_CASE(N)                                                                                   \
  if (n0 == N) {                                                                                       \
    hipLaunchKernelGGL((k_zpass<T, N>), grid, dim3(NT), 0, s, d, op, n1, h, scale);         \
    return hipGetLastError();                                                                          \
  }
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template struct Launch<R>;

}  // namespace ffth
