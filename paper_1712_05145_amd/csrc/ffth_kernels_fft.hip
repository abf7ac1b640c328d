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

template <typename T> int Launch<T>::x_rows(int n, int v) {
#define FFTH_CASE(N) if (n == N) return ffth::xf_rows_v<T>(N, v);
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return 0;
}
template <typename T> int Launch<T>::xi_rows(int n, int v) {
#define FFTH_CASE(N) if (n == N) return ffth::xi_rows_v<T>(N, v);
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return 0;
}
template <typename T> int Launch<T>::y_cols(int n, int v) {
#define FFTH_CASE(N) if (n == N) return ffth::y_cols_v<T>(N, v);
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return 0;
}
template <typename T> int Launch<T>::z_cols(int n, int v) {
#define FFTH_CASE(N) if (n == N) return ffth::z_cols_v<T>(N, v);
  FFTH_ZSIZES(FFTH_CASE)
#undef FFTH_CASE
  return 0;
}

// one launcher per (length, variant): the tile shape is a template argument
// Storage type of the spectrum: full precision, or binary16 (FP32 only)
template <typename T> using Full = C2<T>;

template <typename T, int N, int V, typename S = C2<T>>
static void xfwd_v(bool iso, dim3 grid, hipStream_t s, const Desc* d, int mode, long rows, long nvox) {
  constexpr int RW = ffth::xf_rows_v<T>(N, V), TB = ffth::x_threads_v<T>(N, V);
  constexpr int PL = ffth::plan_of(V);
  if (iso) hipLaunchKernelGGL((k_xfwd<T, N, true, RW, TB, S, PL>), grid, dim3(TB), 0, s, d, mode, rows, nvox);
  else hipLaunchKernelGGL((k_xfwd<T, N, false, RW, TB, S, PL>), grid, dim3(TB), 0, s, d, mode, rows, nvox);
}
template <typename T, int N, int V, typename S = C2<T>>
static void xinv_v(bool iso, dim3 grid, hipStream_t s, const Desc* d, int mode, long rows, long nvox) {
  constexpr int RW = ffth::xi_rows_v<T>(N, V), TB = ffth::xi_threads_v<T>(N, V);
  constexpr int PL = ffth::plan_of(V);
  if (iso) hipLaunchKernelGGL((k_xinv<T, N, true, RW, TB, PL>), grid, dim3(TB), 0, s, d, mode, rows, nvox);
  else hipLaunchKernelGGL((k_xinv<T, N, false, RW, TB, PL>), grid, dim3(TB), 0, s, d, mode, rows, nvox);
}
template <typename T, int N, int V, typename S = C2<T>>
static void xcg3_v(bool iso, dim3 grid, hipStream_t s, const Desc* d, long rows, long nvox) {
  constexpr int RW = ffth::xi_rows_v<T>(N, V), TB = ffth::xi_threads_v<T>(N, V);
  constexpr int PL = ffth::plan_of(V);
  if (iso) hipLaunchKernelGGL((k_xcg3<T, N, true, RW, TB, S, PL>), grid, dim3(TB), 0, s, d, rows, nvox);
  else hipLaunchKernelGGL((k_xcg3<T, N, false, RW, TB, S, PL>), grid, dim3(TB), 0, s, d, rows, nvox);
}
template <typename T, int N, int V, typename S = C2<T>>
static void ypass_v(dim3 grid, hipStream_t s, const Desc* d, int dir, int ncols, int ntiles) {
  constexpr int CW = ffth::y_cols_v<T>(N, V);
  constexpr int TB = ffth::y_threads_v<T>(N, V);
  hipLaunchKernelGGL((k_ypass<T, N, CW, TB, true, 1, S, ffth::plan_of(V)>), grid, dim3(TB), 0, s, d, dir, ncols,
                     ntiles);
}
template <typename T, int N, int V, typename S = C2<T>>
static void zpass_v(dim3 grid, hipStream_t s, const Desc* d, int op, int n1, int h, double scale) {
  constexpr int TK = ffth::z_cols_v<T>(N, V), TB = ffth::z_threads_v<T>(N, V);
  hipLaunchKernelGGL((k_zpass<T, N, TK, TB, true, 1, S, ffth::plan_of(V)>), grid, dim3(TB), 0, s, d, op, n1, h,
                     scale);
}

#define FFTH_VARIANTS_S(F, N, S, ...)        \
  switch (v) {                               \
    case 1: F<T, N, 1, S>(__VA_ARGS__); break; \
    case 2: F<T, N, 2, S>(__VA_ARGS__); break; \
    case 3: F<T, N, 3, S>(__VA_ARGS__); break; \
    case 4: F<T, N, 4, S>(__VA_ARGS__); break; \
    case 5: F<T, N, 5, S>(__VA_ARGS__); break; \
    default: F<T, N, 0, S>(__VA_ARGS__);     \
  }
#define FFTH_VARIANTS(F, N, ...) FFTH_VARIANTS_S(F, N, C2<T>, __VA_ARGS__)
// binary16 instantiations exist for FP32 only
#define FFTH_VARIANTS_H(F, N, ...)                                      \
  if constexpr (std::is_same<T, float>::value) {                        \
    if (h16) {                                                           \
      FFTH_VARIANTS_S(F, N, H2, __VA_ARGS__)                             \
    } else {                                                             \
      FFTH_VARIANTS_S(F, N, C2<T>, __VA_ARGS__)                          \
    }                                                                    \
  } else {                                                               \
    FFTH_VARIANTS_S(F, N, C2<T>, __VA_ARGS__)                            \
  }

template <typename T> hipError_t Launch<T>::xfwd(int n2, bool iso, int v, bool h16, dim3 grid, hipStream_t s,
                                                const Desc* d, int mode, long rows, long nvox) {
#define FFTH_CASE(N)                                                          \
  if (n2 == N) {                                                              \
    FFTH_VARIANTS_H(xfwd_v, N, iso, grid, s, d, mode, rows, nvox)            \
    return hipGetLastError();                                                 \
  }
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template <typename T> hipError_t Launch<T>::xinv(int n2, bool iso, int v, dim3 grid, hipStream_t s, const Desc* d,
                                                int mode, long rows, long nvox) {
#define FFTH_CASE(N)                                                          \
  if (n2 == N) {                                                              \
    FFTH_VARIANTS(xinv_v, N, iso, grid, s, d, mode, rows, nvox)              \
    return hipGetLastError();                                                 \
  }
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template <typename T> hipError_t Launch<T>::xcg3(int n2, bool iso, int v, bool h16, dim3 grid, hipStream_t s,
                                                const Desc* d, long rows, long nvox) {
#define FFTH_CASE(N)                                                          \
  if (n2 == N) {                                                              \
    FFTH_VARIANTS_H(xcg3_v, N, iso, grid, s, d, rows, nvox)                  \
    return hipGetLastError();                                                 \
  }
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template <typename T> hipError_t Launch<T>::ypass(int n1, int v, bool h16, dim3 grid, hipStream_t s, const Desc* d,
                                                 int dir, int ncols, int ntiles) {
#define FFTH_CASE(N)                                                          \
  if (n1 == N) {                                                              \
    FFTH_VARIANTS_H(ypass_v, N, grid, s, d, dir, ncols, ntiles)              \
    return hipGetLastError();                                                 \
  }
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template <typename T> hipError_t Launch<T>::zpass(int n0, int v, bool h16, dim3 grid, hipStream_t s, const Desc* d,
                                                 int op, int n1, int h, double scale) {
#define FFTH_CASE(N)                                                          \
  if (n0 == N) {                                                              \
    FFTH_VARIANTS_H(zpass_v, N, grid, s, d, op, n1, h, scale)                \
    return hipGetLastError();                                                 \
  }
  FFTH_ZSIZES(FFTH_CASE)
#undef FFTH_CASE
  return hipErrorInvalidValue;
}

template <typename T> hipError_t Launch<T>::bicg_finish(dim3 grid, hipStream_t s, const Desc* d, long n) {
  hipLaunchKernelGGL((k_bicg_finish<T>), grid, dim3(NT), 0, s, d, n);
  return hipGetLastError();
}

template <typename T> hipError_t Launch<T>::cg3_finish(dim3 grid, hipStream_t s, const Desc* d, long n) {
  hipLaunchKernelGGL((k_cg3_finish<T>), grid, dim3(NT), 0, s, d, n);
  return hipGetLastError();
}

template struct Launch<R>;

}  // namespace ffth
