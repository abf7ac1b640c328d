// Host-side launchers of the templated FFT-pass kernels: a runtime axis
// length selects the compile-time instantiation.
#pragma once
#include <hip/hip_runtime.h>
#include "ffth_types.h"

// Axis lengths with compiled FFT kernels.
#define FFTH_SIZES(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(256) X(512) X(1024)
// Axis 0 may also have length 1: a 2-D problem in the (x2, x3) plane, whose
// z-pass applies the spectral operator without a transform.
#define FFTH_ZSIZES(X) X(1) FFTH_SIZES(X)

namespace ffth {

bool size_supported(int n);
// every axis length supported (axis 0 may be 1)
bool grid_supported(const int n[3]);

// Every pass has NVAR compiled tile shapes (variant v); the plan picks one
// per pass and precision (autotuned or the default 0).
template <typename T> struct Launch {
  static int x_rows(int n, int v);
  static int xi_rows(int n, int v);
  static int y_cols(int n, int v);
  static int z_cols(int n, int v);
  // h16: spectrum stored as binary16 (FP32 only; the mixed scheme's inner solve)
  static hipError_t xfwd(int n2, bool iso, int v, bool h16, dim3 grid, hipStream_t s, const Desc* d, int mode,
                         long rows, long nvox);
  static hipError_t xinv(int n2, bool iso, int v, dim3 grid, hipStream_t s, const Desc* d, int mode, long rows,
                         long nvox);
  // fused three-term CG iteration (x-inverse, update, x-forward); x-inverse tiles
  static hipError_t xcg3(int n2, bool iso, int v, bool h16, dim3 grid, hipStream_t s, const Desc* d, long rows,
                         long nvox);
  // BiCGSTAB: the pending x update of loads that stopped (n = 6 * voxels)
  static hipError_t bicg_finish(dim3 grid, hipStream_t s, const Desc* d, long n);
  // three-term CG: the last x of loads that stopped after an even iteration
  static hipError_t cg3_finish(dim3 grid, hipStream_t s, const Desc* d, long n);
  static hipError_t ypass(int n1, int v, bool h16, dim3 grid, hipStream_t s, const Desc* d, int dir, int ncols,
                          int ntiles);
  static hipError_t zpass(int n0, int v, bool h16, dim3 grid, hipStream_t s, const Desc* d, int op, int n1, int h,
                          double scale);
};


// non-templated kernels (ffth_kernels_common.hip)
// nblk_i < 0: each entry's own count (Desc::nblk_multi, after a multi-size fused pass)
hipError_t launch_finalize(int nbatch, hipStream_t s, const Desc* d, int op, int nblk_f, int nblk_i);

// Multi-size launches of the FP32 inner iteration (ffth_kernels_multi.hip)
// for grids whose three axis lengths are all in the multi-size set (16, 24,
// 32, 48, 64, 96, 128): one launch per pass over loads of different grids,
// each descriptor carrying its grid (n) and, for the finalize, the block count
// of its fused pass (nblk_multi).  The launch's blocks are listed by the
// segment table sg (one grid per segment, at most MULTI_SEGS; bpd from
// multi_blocks: y, z, fused x blocks per load), grid = sg.off[sg.n] blocks.
bool multi_grid(const int n[3]);
void multi_blocks(const int n[3], int out[3]);
hipError_t multi_ypass(const MultiSegs& sg, hipStream_t s, const Desc* d, int dir, bool h16);
hipError_t multi_zpass(const MultiSegs& sg, hipStream_t s, const Desc* d, int op, bool h16);
hipError_t multi_xcg3(const MultiSegs& sg, hipStream_t s, const Desc* d, bool iso, bool h16);
hipError_t launch_mean_stress(bool iso, int nblk, int nbatch, hipStream_t s, const Desc* d, long nvox);
hipError_t launch_order1_point(bool iso, int nblk, int nbatch, hipStream_t s, const Desc* d, const double* eps0,
                               const double* x1, long nvox);
hipError_t launch_order2_point(bool iso, int nblk, int nbatch, hipStream_t s, const Desc* d, const double* eps1,
                               const double* x1, const double* x2, long nvox);
hipError_t launch_widen(int nbatch, hipStream_t s, const Desc* d, long n);
hipError_t launch_phase_max(hipStream_t s, const uint16_t* phase, long n, int* out);

// text returned by ffth_last_error on this thread (ffth_host.hip)
void set_last_error(const char* msg);

}  // namespace ffth
