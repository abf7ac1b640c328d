// Finalize, volume-average and order-1 pointwise kernels (FP64).
#include "ffth_kernels.h"
#include "ffth_launch.h"

namespace ffth {

__device__ static void fin_check(SolverState* st) {
  const double r = st->res;
  if (!(r == r) || r > 1e6) {
    st->flag = FLAG_DIVERGED;
    st->active = 0;
  } else if (r < st->tol) {
    st->flag = FLAG_CONVERGED;
    st->active = 0;
  } else if (st->iters >= st->max_iter) {
    st->active = 0;  // flag stays RUNNING: not converged
  }
}

// Partial sums are slot-major: part[k * nblk + block].  Each op names how
// many slots of each array it reads.
// Reduction asked of the FP32 inner solve that starts now.  The outer residual
// must still drop by need = 0.8 tol / res (the margin covers the FP32
// round-off of the correction); with at most tmin per solve that takes
// k = ceil(log need / log tmin) more solves, and the reduction is split evenly
// over them: every solve asks for need^(1/k) >= tmin.  Fewer restarts of the
// Krylov iteration than a fixed tmin, and no solve tighter than the sweeps
// still ahead require.
__device__ static double inner_target(double tmin, double outer_tol, double outer_res) {
  if (!(outer_res > 0.0) || !(tmin > 0.0) || !(tmin < 1.0)) return tmin;
  const double need = 0.8 * outer_tol / outer_res;
  if (!(need < 1.0)) return fmax(tmin, 0.5);
  if (need >= tmin) return need;
  const double k = ceil(log(need) / log(tmin));
  return fmax(tmin, pow(need, 1.0 / k));
}

__device__ static void fin_slots(int op, int& nf, int& ni) {
  nf = 0;
  ni = 0;
  switch (op) {
    case FIN_LS_FIRST: nf = 1; ni = 1; break;
    case FIN_BS: ni = 1; break;
    case FIN_RESID_INIT: ni = 2; break;
    case FIN_CG_ALPHA: nf = 1; break;
    case FIN_CG_BETA: ni = 2; break;
    case FIN_OUTER: case FIN_OUTER_P: nf = 1; ni = 2; break;
    case FIN_PROJ: ni = 2; break;
    case FIN_CG3_INIT: nf = 3; break;
    case FIN_CG3: ni = 3; break;
    case FIN_BI_INIT: ni = 1; break;
    case FIN_BI_ALPHA: ni = 1; break;
    case FIN_BI_OMEGA: ni = 5; break;
    case FIN_SUMS_I: case FIN_O1RHS: ni = NRED; break;
  }
}

// This thread's share (i = threadIdx.x mod NT_FIN) of n partials, in a fixed
// order, with 8 independent accumulators so that 8 loads are in flight.
__device__ static double strided_sum(const double* __restrict__ p, int n) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = threadIdx.x;
  for (; i + 7 * NT_FIN < n; i += 8 * NT_FIN) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += p[i + u * NT_FIN];
  }
  for (int u = 0; i < n; i += NT_FIN, ++u) a[u & 7] += p[i];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

__global__ __launch_bounds__(NT_FIN) void k_finalize(const Desc* __restrict__ descs, int op, int nblk_f, int nblk_i) {
  const Desc& d = descs[blockIdx.x];
  SolverState* st = d.st;
  if (!st->active) return;
  if (nblk_i < 0) nblk_i = d.nblk_multi;   // multi-size launch: each entry's own block count
  __shared__ double sf[NRED], si[NRED];
  int nf, ni;
  fin_slots(op, nf, ni);
  double af[NRED], ai[NRED];
#pragma unroll
  for (int k = 0; k < NRED; ++k) {
    af[k] = k < nf ? strided_sum(d.part_f + (long)k * nblk_f, nblk_f) : 0.0;
    ai[k] = k < ni ? strided_sum(d.part_i + (long)k * nblk_i, nblk_i) : 0.0;
  }
  block_sums<NRED, NT_FIN>(af, sf);
  block_sums<NRED, NT_FIN>(ai, si);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double amu = fabs(d.mu0);
  switch (op) {
    case FIN_LS_FIRST: {
      st->nb2 = si[0];
      const double gs = st->gscale > 0.0 ? st->gscale : sqrt(sf[0]) / (2.0 * amu);
      st->iters = 0;
      st->first = 1;
      st->res = 1.0;
      if (sqrt(si[0]) <= st->guard_eps * gs) {
        st->flag = FLAG_ZERO_RHS;
        st->res = 0.0;
        st->active = 0;
      }
      break;
    }
    case FIN_BS:
      st->res = sqrt(si[0] / st->nb2);
      st->iters++;
      st->total++;
      fin_check(st);
      break;
    case FIN_RESID_INIT:
      st->rr = si[1];
      st->res = sqrt(si[0] / st->nb2);
      st->first = 1;
      if (st->res < st->tol) {
        st->flag = FLAG_CONVERGED;
        st->active = 0;
      }
      break;
    case FIN_CG_ALPHA: {
      const double pq = sf[0];
      if (!(pq > 0.0) || !(st->rr == st->rr)) {
        st->flag = FLAG_DIVERGED;
        st->active = 0;
      } else {
        st->alpha = st->rr / pq;
      }
      break;
    }
    case FIN_CG_BETA:
      st->res = sqrt(si[1] / st->nb2);
      st->iters++;
      st->total++;
      st->beta = si[0] / st->rr;
      st->rr = si[0];
      st->first = 0;
      fin_check(st);
      break;
    case FIN_CG3_INIT: {
      // three-term CG: rho_0 = <r,r>_C0, mu_0 = <r,Ar>_C0, gamma_0 = rho_0 / mu_0, omega_0 = 1
      if (!(sf[1] > 0.0) || !(sf[0] > 0.0)) {
        st->flag = sf[0] > 0.0 ? FLAG_DIVERGED : FLAG_CONVERGED;
        st->active = 0;
        break;
      }
      st->rr = sf[0];
      st->alpha = sf[0] / sf[1];
      st->beta = 1.0;
      st->alpha_prev = 0.0;
      st->beta_prev = 1.0;
      st->xpend = 0;
      st->best_res = 1.0;
      st->best_it = 0;
      st->stalled = 0;
      st->first = 1;
      break;
    }
    case FIN_CG3: {
      // si = (rho_{k+1}, mu_{k+1}, ||r_{k+1}||^2); state holds rho_k, gamma_k, omega_k
      st->res = sqrt(si[2] / st->nb2);
      st->iters++;
      st->total++;
      const double g = si[0] / si[1];
      const double den = 1.0 - (g / st->alpha) * (si[0] / st->rr) / st->beta;
      const double om = 1.0 / den;
      st->first = 0;
      // stop before the scalars advance: a solve that stops keeps gamma_k,
      // omega_k (and gamma_{k-1}, omega_{k-1}) of its last iteration k, from
      // which k_cg3_finish forms x_{k+1} when k was even
      if (st->res < st->tol) {
        st->flag = FLAG_CONVERGED;
        st->active = 0;
      } else if (!(si[1] > 0.0) || !(om == om) || !(fabs(om) < 1e6) || !(st->res == st->res) || st->res > 1e6) {
        st->flag = FLAG_DIVERGED;
        st->active = 0;
      } else if (st->total >= st->max_iter) {
        // iteration budget (over all solves sharing the state: the mixed
        // scheme's inner solves count together) spent; flag stays RUNNING
        st->active = 0;
      } else if (st->iters - st->best_it >= CG3_STALL && !(st->res < st->best_res)) {
        // no new smallest residual for CG3_STALL iterations: the rounding
        // floor of this precision; flag stays RUNNING
        st->stalled = 1;
        st->active = 0;
      } else {
        st->rr = si[0];
        st->alpha_prev = st->alpha;
        st->beta_prev = st->beta;
        st->alpha = g;
        st->beta = om;
      }
      if (st->res < st->best_res) {
        st->best_res = st->res;
        st->best_it = st->iters;
      }
      // x is formed on odd iterations: after an even last one (iters odd) it is owed
      if (!st->active) st->xpend = st->iters & 1;
      break;
    }
    case FIN_BI_INIT:
      // BiCGSTAB start: r_0 = b - A b, rho = <r^, r_0> = ||r_0||^2
      st->rr = si[0];
      st->res = sqrt(si[0] / st->nb2);
      st->alpha = st->omega = 1.0;
      st->beta = 0.0;
      st->first = 1;
      st->pending = 0;
      if (st->res < st->tol) {
        st->flag = FLAG_CONVERGED;
        st->active = 0;
      }
      break;
    case FIN_BI_ALPHA: {
      // alpha = rho / <r^, v>; the previous x update is applied by now
      st->pending = 0;
      const double rv = si[0];
      if (!(fabs(rv) > 0.0) || !(rv == rv)) {
        st->flag = FLAG_DIVERGED;
        st->active = 0;
      } else {
        st->alpha = st->rr / rv;
      }
      break;
    }
    case FIN_BI_OMEGA: {
      // si = (<t,s>, <t,t>, <r^,s>, <r^,t>, <s,s>)
      const double ts = si[0], tt = si[1];
      const double om = tt > 0.0 ? ts / tt : 0.0;
      const double rho = si[2] - om * si[3];
      const double r2 = fmax(0.0, si[4] - 2.0 * om * ts + om * om * tt);   // ||s - omega t||^2
      st->omega = om;
      st->pending = 1;
      st->first = 0;
      st->iters++;
      st->total++;
      st->res = sqrt(r2 / st->nb2);
      if (st->res < st->tol) {
        st->flag = FLAG_CONVERGED;
        st->active = 0;
      } else if (!(om != 0.0) || !(rho == rho) || !(fabs(rho) > 0.0)) {
        st->flag = FLAG_DIVERGED;   // breakdown
        st->active = 0;
      } else {
        st->beta = (rho / st->rr) * (st->alpha / om);
        st->rr = rho;
        fin_check(st);
      }
      break;
    }
    case FIN_PROJ: {
      // compatible part of the FP64 residual: restart the FP32 inner solve on it
      SolverState* in = d.st2;
      st->proj++;
      in->tol = inner_target(in->tol0, st->tol, st->res);
      in->active = si[0] > 0.0 ? 1 : 0;
      in->nb2 = si[0];
      in->dscale = si[0] > 0.0 ? sqrt(si[0] * d.inv_nvox) : 1.0;
      in->rr = si[1];
      in->first = 1;
      in->iters = 0;
      in->xpend = 0;
      in->flag = FLAG_RUNNING;
      in->res = 1.0;
      break;
    }
    case FIN_OUTER:
    case FIN_OUTER_P: {
      SolverState* in = d.st2;
      if (st->iters == 0) {
        st->nb2 = si[0];
        const double gs = st->gscale > 0.0 ? st->gscale : sqrt(sf[0]) / (2.0 * amu);
        if (sqrt(si[0]) <= st->guard_eps * gs) {
          st->flag = FLAG_ZERO_RHS;
          st->res = 0.0;
          st->active = 0;
          in->active = 0;
          break;
        }
      }
      st->res = sqrt(si[0] / st->nb2);
      st->iters++;
      st->fp64_apps++;
      if (!(st->res == st->res) || st->res > 1e6) {
        st->flag = FLAG_DIVERGED;
        st->active = 0;
      } else if (st->res < st->tol) {
        st->flag = FLAG_CONVERGED;
        st->active = 0;
      } else if (st->iters >= st->max_iter) {
        st->active = 0;
      }
      if (!st->active) {
        in->active = 0;
      } else if (op == FIN_OUTER_P) {
        in->active = 0;  // the projection pass sets the inner solve up
      } else {
        in->active = 1;
        in->tol = inner_target(in->tol0, st->tol, st->res);
        in->nb2 = si[0];
        in->dscale = si[0] > 0.0 ? sqrt(si[0] * d.inv_nvox) : 1.0;
        in->rr = si[1];
        in->first = 1;
        in->iters = 0;
        in->xpend = 0;
        in->flag = FLAG_RUNNING;
        in->res = 1.0;
      }
      break;
    }
    case FIN_SUMS_I:
      for (int k = 0; k < NRED; ++k) st->sums[k] = si[k];
      break;
    case FIN_O1RHS:
      for (int k = 0; k < NRED; ++k) st->sums[k] = si[k];
      st->gscale = (sqrt(si[0]) + sqrt(si[1])) / (2.0 * amu);
      break;
  }
}

template <bool ISO>
__global__ __launch_bounds__(NT) void k_mean_stress(const Desc* __restrict__ descs, long nvox) {
  const Desc& d = descs[blockIdx.y];
  if (!d.st->active) return;
  double acc[NRED] = {0, 0, 0, 0, 0, 0, 0, 0};
  const double* x = (const double*)d.x;
  for (long vox = (long)blockIdx.x * NT + threadIdx.x; vox < nvox; vox += (long)gridDim.x * NT) {
    const int ph = d.phase[vox];
    double e[6], s[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) e[c] = x[c * nvox + vox] + (d.P ? 0.0 : d.E[c]);
    apply_mat<double, ISO>(d.mat64, ph, false, e, s);
    if (d.P) {
#pragma unroll
      for (int c = 0; c < 6; ++c) s[c] += d.P[c * nvox + vox];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += s[c];
  }
  block_sums<NRED, NT>(acc, d.part_i + blockIdx.x, gridDim.x);
}

template <bool ISO>
__global__ __launch_bounds__(NT) void k_order1_point(const Desc* __restrict__ descs, const double* __restrict__ eps0,
                                                     const double* __restrict__ x1, long nvox) {
  const Desc& d = descs[blockIdx.y];
  if (!d.st->active) return;
  double acc[NRED] = {0, 0, 0, 0, 0, 0, 0, 0};
  double* pout = (double*)d.io;   // [6][N] p_2
  double* gout = (double*)d.p;    // [3][N] g
  const double mult[6] = {1, 1, 1, 2, 2, 2};
  for (long vox = (long)blockIdx.x * NT + threadIdx.x; vox < nvox; vox += (long)gridDim.x * NT) {
    const int ph = d.phase[vox];
    double xg[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double g[3] = {0, 0, 0};
#pragma unroll
    for (int J = 0; J < 6; ++J) {
      const double cj = mult[J];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double xv = cj * x1[(long)(J * 3 + m) * nvox + vox];
#pragma unroll
        for (int j = 0; j < 3; ++j) xg[m][j] += xv * d.G[J * 3 + j];
      }
      // S^J = C : (E^J + eps^J), E^J the unit engineering load J as a tensor
      double e[6], s[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = eps0[((long)J * 6 + c) * nvox + vox] + (c == J ? (J < 3 ? 1.0 : 0.5) : 0.0);
      apply_mat<double, ISO>(d.mat64, ph, false, e, s);
      // full matrix rows of S from (11,22,33,23,13,12)
      const double S[3][3] = {{s[0], s[5], s[4]}, {s[5], s[1], s[3]}, {s[4], s[3], s[2]}};
#pragma unroll
      for (int i = 0; i < 3; ++i)
        g[i] += cj * (S[i][0] * d.G[J * 3 + 0] + S[i][1] * d.G[J * 3 + 1] + S[i][2] * d.G[J * 3 + 2]);
    }
    double sy[6] = {xg[0][0], xg[1][1], xg[2][2], 0.5 * (xg[1][2] + xg[2][1]), 0.5 * (xg[0][2] + xg[2][0]),
                    0.5 * (xg[0][1] + xg[1][0])};
    double p2[6];
    apply_mat<double, ISO>(d.mat64, ph, false, sy, p2);
#pragma unroll
    for (int c = 0; c < 6; ++c) pout[c * nvox + vox] = p2[c];
#pragma unroll
    for (int i = 0; i < 3; ++i) gout[i * nvox + vox] = g[i];
    acc[0] += frob_w(p2, p2);
    acc[1] += g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    acc[2] += g[0];
    acc[3] += g[1];
    acc[4] += g[2];
  }
  block_sums<NRED, NT>(acc, d.part_i + blockIdx.x, gridDim.x);
}

// Order 2 (the paper's alpha = 3): per voxel, from the order-0 corrector
// displacements x1 [6][3][N], the 18 order-1 unit-gradient strains eps1
// [18][6][N] and their displacements x2 [18][3][N]:
//   V_am = sum_{J,j} x2[J,j]_a H[J,j,m],  p_3 = C : sym(V)
//   S_2^(J,j) = C : (eps1[J,j] + sym(c_J x1[J] x e_j)),  g_i = sum_{J,j,m} S_2^(J,j)_im H[J,j,m]
template <bool ISO>
__global__ __launch_bounds__(NT) void k_order2_point(const Desc* __restrict__ descs, const double* __restrict__ eps1,
                                                     const double* __restrict__ x1, const double* __restrict__ x2,
                                                     long nvox) {
  const Desc& d = descs[blockIdx.y];
  if (!d.st->active) return;
  double acc[NRED] = {0, 0, 0, 0, 0, 0, 0, 0};
  double* pout = (double*)d.io;   // [6][N] p_3
  double* gout = (double*)d.p;    // [3][N] g
  const double mult[6] = {1, 1, 1, 2, 2, 2};
  for (long vox = (long)blockIdx.x * NT + threadIdx.x; vox < nvox; vox += (long)gridDim.x * NT) {
    const int ph = d.phase[vox];
    double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double g[3] = {0, 0, 0};
    for (int jj = 0; jj < 18; ++jj) {
      const int J = jj / 3, j = jj % 3;
      const double h0 = d.H[jj * 3 + 0], h1 = d.H[jj * 3 + 1], h2 = d.H[jj * 3 + 2];
      if (h0 == 0.0 && h1 == 0.0 && h2 == 0.0) continue;   // the same for every thread of the load
      double xe[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double w = x2[((long)jj * 3 + a) * nvox + vox];
        V[a][0] += w * h0;
        V[a][1] += w * h1;
        V[a][2] += w * h2;
        xe[a] = mult[J] * x1[((long)J * 3 + a) * nvox + vox];
      }
      // eps1 + sym(xe x e_j) in tensor components (11,22,33,23,13,12)
      double e[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = eps1[((long)jj * 6 + c) * nvox + vox];
      if (j == 0) { e[0] += xe[0]; e[5] += 0.5 * xe[1]; e[4] += 0.5 * xe[2]; }
      else if (j == 1) { e[1] += xe[1]; e[5] += 0.5 * xe[0]; e[3] += 0.5 * xe[2]; }
      else { e[2] += xe[2]; e[4] += 0.5 * xe[0]; e[3] += 0.5 * xe[1]; }
      double s[6];
      apply_mat<double, ISO>(d.mat64, ph, false, e, s);
      const double S[3][3] = {{s[0], s[5], s[4]}, {s[5], s[1], s[3]}, {s[4], s[3], s[2]}};
#pragma unroll
      for (int i = 0; i < 3; ++i) g[i] += S[i][0] * h0 + S[i][1] * h1 + S[i][2] * h2;
    }
    double sy[6] = {V[0][0], V[1][1], V[2][2], 0.5 * (V[1][2] + V[2][1]), 0.5 * (V[0][2] + V[2][0]),
                    0.5 * (V[0][1] + V[1][0])};
    double p3[6];
    apply_mat<double, ISO>(d.mat64, ph, false, sy, p3);
#pragma unroll
    for (int c = 0; c < 6; ++c) pout[c * nvox + vox] = p3[c];
#pragma unroll
    for (int i = 0; i < 3; ++i) gout[i * nvox + vox] = g[i];
    acc[0] += frob_w(p3, p3);
    acc[1] += g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    acc[2] += g[0];
    acc[3] += g[1];
    acc[4] += g[2];
  }
  block_sums<NRED, NT>(acc, d.part_i + blockIdx.x, gridDim.x);
}

__global__ void k_widen(const Desc* __restrict__ descs, long n) {
  const Desc& d = descs[blockIdx.y];
  const float* src = (const float*)d.x;
  double* dst = (double*)d.out;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

__global__ void k_phase_max(const uint16_t* __restrict__ phase, long n, int* out) {
  int m = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    m = max(m, (int)phase[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

template __global__ void k_mean_stress<true>(const Desc*, long);
template __global__ void k_mean_stress<false>(const Desc*, long);
template __global__ void k_order1_point<true>(const Desc*, const double*, const double*, long);
template __global__ void k_order1_point<false>(const Desc*, const double*, const double*, long);
template __global__ void k_order2_point<true>(const Desc*, const double*, const double*, const double*, long);
template __global__ void k_order2_point<false>(const Desc*, const double*, const double*, const double*, long);

}  // namespace ffth

namespace ffth {

bool size_supported(int n) {
#define FFTH_CASE(N) if (n == N) return true;
  FFTH_SIZES(FFTH_CASE)
#undef FFTH_CASE
  return false;
}

bool grid_supported(const int n[3]) {
  return (n[0] == 1 || size_supported(n[0])) && size_supported(n[1]) && size_supported(n[2]);
}

hipError_t launch_finalize(int nbatch, hipStream_t s, const Desc* d, int op, int nblk_f, int nblk_i) {
  hipLaunchKernelGGL(k_finalize, dim3(nbatch), dim3(NT_FIN), 0, s, d, op, nblk_f, nblk_i);
  return hipGetLastError();
}

hipError_t launch_mean_stress(bool iso, int nblk, int nbatch, hipStream_t s, const Desc* d, long nvox) {
  if (iso) hipLaunchKernelGGL(k_mean_stress<true>, dim3(nblk, nbatch), dim3(NT), 0, s, d, nvox);
  else hipLaunchKernelGGL(k_mean_stress<false>, dim3(nblk, nbatch), dim3(NT), 0, s, d, nvox);
  return hipGetLastError();
}

hipError_t launch_order1_point(bool iso, int nblk, int nbatch, hipStream_t s, const Desc* d, const double* eps0,
                               const double* x1, long nvox) {
  if (iso) hipLaunchKernelGGL(k_order1_point<true>, dim3(nblk, nbatch), dim3(NT), 0, s, d, eps0, x1, nvox);
  else hipLaunchKernelGGL(k_order1_point<false>, dim3(nblk, nbatch), dim3(NT), 0, s, d, eps0, x1, nvox);
  return hipGetLastError();
}

hipError_t launch_order2_point(bool iso, int nblk, int nbatch, hipStream_t s, const Desc* d, const double* eps1,
                               const double* x1, const double* x2, long nvox) {
  if (iso) hipLaunchKernelGGL(k_order2_point<true>, dim3(nblk, nbatch), dim3(NT), 0, s, d, eps1, x1, x2, nvox);
  else hipLaunchKernelGGL(k_order2_point<false>, dim3(nblk, nbatch), dim3(NT), 0, s, d, eps1, x1, x2, nvox);
  return hipGetLastError();
}

hipError_t launch_phase_max(hipStream_t s, const uint16_t* phase, long n, int* out) {
  hipLaunchKernelGGL(k_phase_max, dim3(512), dim3(256), 0, s, phase, n, out);
  return hipGetLastError();
}

hipError_t launch_widen(int nbatch, hipStream_t s, const Desc* d, long n) {
  hipLaunchKernelGGL(k_widen, dim3(1024, nbatch), dim3(256), 0, s, d, n);
  return hipGetLastError();
}

}  // namespace ffth
