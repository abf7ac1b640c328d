// Plain-old-data structures shared by the host driver and the kernels.
#pragma once
#include <stdint.h>

namespace ffth {

// Per-load iteration state, resident in device memory.  The finalize kernel
// is its only writer while a solve runs; the host reads it every few
// iterations to decide whether to keep launching.
struct SolverState {
  double tol;        // relative residual to reach
  double nb2;        // ||b||^2, the reference of the relative residual
  double rr;         // CG: <r, r>_C0
  double alpha, beta;  // CG: step and direction coefficients; three-term CG: gamma and omega
  double res;        // last relative residual
  double gscale;     // strain-like scale of the zero right-hand-side guard (<= 0: from ||P||)
  double guard_eps;  // relative threshold of the guard
  double sums[8];    // last finalized block sums (diagnostics, mean stress)
  int32_t active;    // 1 while the load iterates; every kernel skips inactive loads
  int32_t iters;     // iterations of the current solve
  int32_t total;     // iterations over all solves sharing this state
  int32_t flag;      // FLAG_*
  int32_t first;     // CG: the next direction update takes p = r
  int32_t max_iter;  // stop (unconverged) after this many iterations
  int32_t fp64_apps; // FP64 operator applications (outer state only)
  int32_t proj;      // FP32 projection passes (outer state only)
  double omega;      // BiCGSTAB: omega of the last iteration
  double dscale;     // inner state: RMS of the inner right-hand side (binary16 spectrum scale)
  int32_t pending;   // BiCGSTAB: x += alpha p + omega s of the last iteration not applied yet
  int32_t xpend;     // three-term CG: stopped after an even iteration, x of the last one not formed yet
  double tol0;       // inner state: the tightest reduction asked of one inner solve
  double alpha_prev, beta_prev;  // three-term CG: gamma and omega of the iteration before the current one
  double best_res;   // three-term CG: smallest residual of the current solve
  int32_t best_it;   // three-term CG: iteration that reached it
  int32_t stalled;   // three-term CG: the solve stopped without a new smallest residual for CG3_STALL iterations
};

// Three-term CG stops a solve whose recursive residual set no new minimum in
// this many iterations (its rounding floor: an FP32 inner solve asked for more
// than its arithmetic reaches hands over to the FP64 sweep instead).
constexpr int CG3_STALL = 64;

enum : int32_t { FLAG_RUNNING = 0, FLAG_CONVERGED = 1, FLAG_DIVERGED = 2, FLAG_ZERO_RHS = 3 };

// Everything a kernel needs about one batch entry (one load case of one
// RVE).  Kernels index an array of these with blockIdx.y (blockIdx.x for the
// one-block-per-entry kernels).
struct Desc {
  const uint16_t* phase;   // [N] phase ids
  const double* mat64;     // per phase: iso (lam, mu, lam-lam0, mu-mu0) or gen (M[36], M-M0[36])
  const float* mat32;
  void* x;                 // iterate (compute precision)
  void* r;                 // residual (compute precision, or FP32 when r_f32)
  void* p;                 // CG search direction
  float* delta;            // FP32 correction fused into the FP64 residual pass (or null)
  float* delta1;           // its second slot when the inner solve is the three-term CG (or null)
  void* x1;                // three-term CG: second iterate slot (x_{k-1}, overwritten by x_{k+1})
  void* r1;                // three-term CG: second residual slot (r_k in slot k mod 2)
  void* rh;                // BiCGSTAB: shadow residual r^ = r_0
  void* v;                 // BiCGSTAB: v = A p
  void* s;                 // BiCGSTAB: s = r - alpha v
  void* t;                 // BiCGSTAB: t = A s
  const double* P;         // stored right-hand-side polarization [6][N] (or null: C:E)
  void* io;                // generic input field (copy-in mode; order-1 p_2 output)
  void* out;               // generic output field (store / accumulate modes)
  void* spec;              // half spectrum [n0][n1][n2/2][6] complex
  void* spec2;             // binary16 inner solve: FP32 copy after the spectral operator
  double* part_f;          // [nblk][8] block sums of the forward x-pass
  double* part_i;          // [nblk][8] block sums of the inverse x-pass / pointwise kernels
  SolverState* st;         // gating state
  SolverState* st2;        // secondary state (outer -> inner set-up)
  double lam0, mu0;        // reference medium of this entry's problem
  double E[6];             // macroscopic strain, tensor components
  double G[18];            // order-1 gradient load G[J*3 + j]
  double H[54];            // order-2 load H[J*9 + j*3 + m] = d^2 E_J / dY_j dY_m
  double inv_nvox;         // 1 / voxels
  double tau_scale;        // binary16 spectrum: factor on the polarization before the x-transform
  double op_scale;         // binary16 spectrum: factor of the spectral operator (replaces 1/N)
  int32_t nc;              // components of io (3 or 6) read by the copy-in x-pass
  int32_t r_f32;           // residual stored as FP32
  int32_t h16;             // the inner solve keeps its spectrum in binary16
  int32_t nc_out;          // components of out written by the store / accumulate x-pass (0: nc)
  int32_t delta_gate;      // delta is the three-term inner solve's x: absent while it has no iteration
  int32_t n[3];            // grid of this entry (multi-size launches)
  int32_t nblk_multi;      // partial-sum blocks of its multi-size fused pass (finalize with nblk_i < 0)
  int32_t x_zero;          // the iterate x is zero (first residual sweep of a solve): not read
};

// x-pass (forward) modes
enum : int32_t { XF_LS = 0, XF_MATVEC = 1, XF_CG = 2, XF_COPY = 3, XF_C0 = 4, XF_R3 = 5, XF_BI1 = 6, XF_BI2 = 7 };
// x-pass (inverse) modes
enum : int32_t {
  XI_STORE = 0, XI_ACCUM = 1, XI_BS = 2, XI_RESID = 3, XI_BS_INNER = 4, XI_CG = 5, XI_PROJ = 6, XI_BI1 = 7, XI_BI2 = 8
};
// spectral operators of the z-pass
enum : int32_t { OP_GAMMA = 0, OP_THETA = 1, OP_DISP = 2 };
// finalize operations
enum : int32_t {
  FIN_LS_FIRST = 0, FIN_BS = 1, FIN_RESID_INIT = 2, FIN_CG_ALPHA = 3, FIN_CG_BETA = 4,
  FIN_OUTER = 5, FIN_SUMS_I = 6, FIN_O1RHS = 7, FIN_OUTER_P = 8, FIN_PROJ = 9, FIN_CG3_INIT = 10, FIN_CG3 = 11,
  FIN_BI_INIT = 12, FIN_BI_ALPHA = 13, FIN_BI_OMEGA = 14
};

// Block list of a multi-size launch: loads of one grid form a segment of
// consecutive descriptors (first .. first + count - 1), each taking bpd
// blocks padded to a multiple of 8 (the XCDs); segment s owns the launch's
// blocks [off[s], off[s + 1]).
constexpr int MULTI_SEGS = 16;
struct MultiSegs {
  int32_t n;
  int32_t first[MULTI_SEGS];
  int32_t bpd[MULTI_SEGS];
  int32_t off[MULTI_SEGS + 1];
};

constexpr int NRED = 8;   // doubles per block in the partial-sum arrays
constexpr int NVAR = 6;   // compiled tile shapes / radix plans per pass (autotuner candidates)

}  // namespace ffth
