// HIP kernels of one iteration of the Moulinec-Suquet Basic Scheme / its CG
// form (Algorithm 1 and eq. (6) of arXiv:1712.05145), organised as five
// HBM-streaming passes over a half spectrum (k2 < n2/2, six interleaved
// components) stored k2-chunked as [k2 / KC][n0][n1][k2 % KC][6] complex,
// KC = kchunk(n2/2) (at most 16): every z-column then strides KC*6*n1
// complex values between rows instead of a whole plane:
//
//   x-pass (forward)   constitutive law / polarization tau (Algorithm 1, first
//                      step; eq. (2)) fused with the real-to-complex FFT along
//                      the contiguous axis (two real components per complex FFT)
//   y-pass             complex FFT along axis 1 (forward or inverse)
//   z-pass             forward FFT along axis 0, the spectral operator (Green
//                      operator below eq. (5) with eta_hat(0) = 0; theta of
//                      eq. (12); displacement recovery from eq. (1)), inverse FFT
//   y-pass (inverse)
//   x-pass (inverse)   complex-to-real FFT fused with the Basic Scheme / CG
//                      update and the residual reductions
//
// All FFTs run in LDS (mixed-radix Stockham, fft_device.h).  Block tile
// sizes are compile-time functions of the axis length and precision.
#pragma once
#include <type_traits>

#include "fft_device.h"
#include "ffth_types.h"

namespace ffth {

constexpr int NT = 256;   // threads per block of every FFT pass

constexpr int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
// Tile shapes and block sizes, chosen from a sweep of every pass at 256^3 on
// MI355X (rows per x-pass block, interleaved columns per y/z block, threads).
template <typename T> constexpr int x_rows(int n) {          // forward x-pass
  int r = 512 / n;
  return r < 1 ? 1 : pow2_floor(r);
}
template <typename T> constexpr int xi_rows(int n) {         // inverse x-pass
  int r = (sizeof(T) == 4 ? 256 : 512) / n;
  return r < 1 ? 1 : pow2_floor(r);
}
template <typename T> constexpr int y_cols(int n) {
  int c = (sizeof(T) == 4 ? 4096 : 2048) / n;
  int cap = sizeof(T) == 4 ? 16 : 8;
  c = c > cap ? cap : c;
  return c < 1 ? 1 : pow2_floor(c);
}
template <typename T> constexpr int y_threads(int n) { return sizeof(T) == 4 && n >= 128 ? 512 : 256; }
template <typename T> constexpr int z_cols(int n) {
  int c = 256 / n;
  c = c > 16 ? 16 : c;
  return c < 1 ? 1 : pow2_floor(c);
}
// Candidate shapes for the runtime autotuner: variant 0 is the measured
// default above, 1 and 2 halve / double the tile (or swap the block size of
// the y-pass), within 96 KB of LDS per block; 3 keeps the x tile of 0 with one
// wave per block (lengths whose Stockham stages have fewer butterflies than
// the default block has threads; for the inverse and fused x-passes, whose
// default is often one row, variant 1 is then two rows with 512 threads).
// The z-pass takes twice the columns (1),
// four times with 512 threads (2) or three times with 512 threads (3): rows
// of >= 144 contiguous bytes in FP32.  Variants 4 and 5 keep the default
// tile and change the radix plan of the transform (fft_device.h).
template <typename T> constexpr int lds_cap_rows(int n) {          // x-pass rows within 96 KB
  int r = 98304 / (3 * (n + n / 16) * (int)(2 * sizeof(T)));
  return r < 1 ? 1 : pow2_floor(r);
}
template <typename T> constexpr int var_rows(int r0, int n, int v) {
  int r = v == 1 ? (r0 > 1 ? r0 / 2 : 1) : v == 2 ? 2 * r0 : r0;   // v == 3: r0
  int c = lds_cap_rows<T>(n);
  return r > c ? c : r;
}
template <typename T> constexpr int xf_rows_v(int n, int v) { return var_rows<T>(x_rows<T>(n), n, v); }
// inverse / fused x-pass: variant 1 of a one-row tile (nothing to halve)
// doubles the rows with 512 threads instead
template <typename T> constexpr bool xi_wide_v(int n, int v) {
  return v == 1 && xi_rows<T>(n) == 1 && lds_cap_rows<T>(n) >= 2;
}
template <typename T> constexpr int xi_rows_v(int n, int v) {
  return xi_wide_v<T>(n, v) ? 2 : var_rows<T>(xi_rows<T>(n), n, v);
}
template <typename T> constexpr int y_cols_v(int n, int v) {
  int c = y_cols<T>(n);
  if (v == 2) c = c > 1 ? c / 2 : 1;
  return c;
}
template <typename T> constexpr int x_threads_v(int, int v) { return v == 3 ? 64 : NT; }
template <typename T> constexpr int z_threads_v(int, int v) { return v == 2 || v == 3 ? 512 : NT; }
// variants 4 and 5: the default tile shape (variant 0) with radix plans 1 and 2
constexpr int plan_of(int v) { return v >= 4 ? v - 3 : 0; }
template <typename T> constexpr int xi_threads_v(int n, int v) { return xi_wide_v<T>(n, v) ? 512 : x_threads_v<T>(n, v); }
template <typename T> constexpr int y_threads_v(int n, int v) {
  return v == 1 ? (y_threads<T>(n) == 512 ? 256 : 512) : v == 2 ? 256 : y_threads<T>(n);
}
template <typename T> constexpr int z_cols_v(int n, int v) {
  int c = z_cols<T>(n);
  c = v == 1 ? 2 * c : v == 2 ? 4 * c : v == 3 ? 3 * c : c;
  const int cap = 98304 / (n * 6 * (int)(2 * sizeof(T)));
  c = c > cap ? (cap < 1 ? 1 : pow2_floor(cap)) : c;
  return c;
}

// k2 values per chunk of the half-spectrum layout: largest divisor of h up to 16
__host__ __device__ constexpr int kchunk(int h) {
  int c = h < 16 ? h : 16;
  while (h % c) --c;
  return c;
}
// index of (row = i0*n1 + i1, k2, component c) in the chunked half spectrum
__device__ __forceinline__ long spec_at(long row, int k2, int c, long rows, int kc) {
  return ((long)(k2 / kc) * rows + row) * (kc * 6) + (k2 % kc) * 6 + c;
}

// vector width of LDS / global accesses in the y and z passes (1: measured
// faster than 16-byte pairs, which halve the threads busy in each stage)
template <typename T> constexpr int vec_width() { return 1; }

// ---------------------------------------------------------------------------
// Constitutive law helpers.  Tensor-component vectors (11,22,33,23,13,12).
// Isotropic table row: (lam, mu, lam - lam0, mu - mu0).  Generic table row:
// M (36, maps tensor components to stress) followed by M - M0 (36).
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ const T* mat_of(const Desc& d);
template <> __device__ __forceinline__ const float* mat_of<float>(const Desc& d) { return d.mat32; }
template <> __device__ __forceinline__ const double* mat_of<double>(const Desc& d) { return d.mat64; }

// out = (C or C - C0)(phase) : e
template <typename T, bool ISO>
__device__ __forceinline__ void apply_mat(const T* mat, int ph, bool delta, const T (&e)[6], T (&out)[6]) {
  if constexpr (ISO) {
    const T lam = mat[ph * 4 + (delta ? 2 : 0)];
    const T mu2 = T(2) * mat[ph * 4 + (delta ? 3 : 1)];
    const T tr = e[0] + e[1] + e[2];
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = mu2 * e[c] + (c < 3 ? lam * tr : T(0));
  } else {
    const T* m = mat + ph * 72 + (delta ? 36 : 0);
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      T s = 0;
#pragma unroll
      for (int b = 0; b < 6; ++b) s += m[a * 6 + b] * e[b];
      out[a] = s;
    }
  }
}

template <typename T> __device__ __forceinline__ T frob_w(const T (&a)[6], const T (&b)[6]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + T(2) * (a[3] * b[3] + a[4] * b[4] + a[5] * b[5]);
}
// a : b (off-diagonal tensor components counted twice) accumulated in FP64
template <typename T> __device__ __forceinline__ double frob_d(const T (&a)[6], const T (&b)[6]) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) s += (c < 3 ? 1.0 : 2.0) * (double)a[c] * (double)b[c];
  return s;
}
// a : b for a block sum: FP32 operands are multiplied in FP64 (products of
// small residuals would underflow in FP32); FP64 keeps frob_w's order
template <typename T> __device__ __forceinline__ double frob_acc(const T (&a)[6], const T (&b)[6]) {
  if constexpr (sizeof(T) == 4) return frob_d(a, b);
  else return frob_w(a, b);
}
// C0 inner product density lam0 tr a tr b + 2 mu0 a:b
__device__ __forceinline__ double c0_ip(double lam0, double mu0, const double (&a)[6], const double (&b)[6]) {
  const double ta = a[0] + a[1] + a[2], tb = b[0] + b[1] + b[2];
  const double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + 2.0 * (a[3] * b[3] + a[4] * b[4] + a[5] * b[5]);
  return lam0 * ta * tb + 2.0 * mu0 * ab;
}

// Residual slot of iteration k in the three-term CG: r_k sits in slot k mod 2
// (r_{k+1} overwrites r_{k-1}, which iteration k reads first).
__device__ __forceinline__ void* rslot(const Desc& d, int k) { return (k & 1) ? d.r1 : d.r; }

// ---------------------------------------------------------------------------
// x-pass, forward: polarization + real-to-complex FFT along axis 2.
// ---------------------------------------------------------------------------
// MI355X dispatches the blocks of a grid round-robin over its 8 XCDs (each
// with its own L2).  Renumbering so that each XCD walks a contiguous range of
// tiles keeps neighbouring tiles, which share cache lines at tile edges, in
// the same L2 at about the same time.
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  constexpr int NX = 8;
  const int q = nblk / NX, r = nblk % NX;
  const int x = bid % NX, i = bid / NX;
  return x * q + (x < r ? x : r) + i;
}

// Rows of the x-passes sit in LDS as 3 complex sequences per row, each
// packing two real components (c = 2q, 2q + 1) as real and imaginary part,
// so that one complex FFT transforms two real rows.

// After a forward FFT: unpack the two real transforms of each sequence and
// store the half spectrum (k2 < N2/2) of the block's rows.
template <typename T, int N2, int ROWS, int NTB, typename S = C2<T>>
__device__ __forceinline__ void store_rows_r2c(S* spec, const C2<T>* z, long row0, long rows_total) {
  constexpr int RS = N2 + N2 / 16;
  constexpr int H = N2 / 2;
  for (int v = threadIdx.x; v < ROWS * H * 6; v += NTB) {
    const int rr = v / (H * 6), rem = v % (H * 6);
    const long row = row0 + rr;
    if (row >= rows_total) continue;
    const int k = rem / 6, c = rem % 6, q = c >> 1;
    const C2<T>* zr = z + (rr * 3 + q) * RS;
    const C2<T> z1 = zr[padx<true>(k)];
    const C2<T> z2 = conj(zr[padx<true>((N2 - k) % N2)]);
    C2<T> o;
    if ((c & 1) == 0) o = (z1 + z2) * T(0.5);
    else o = C2<T>{(z1.y - z2.y) * T(0.5), -(z1.x - z2.x) * T(0.5)};
    sstore<T>(spec + spec_at(row, k, c, rows_total, kchunk(H)), o);
  }
}

// Before an inverse FFT: load the half spectrum of the block's rows and
// rebuild the full Hermitian-packed sequences (Nyquist bin zero).
template <typename T, int N2, int ROWS, int NTB, typename S = C2<T>>
__device__ __forceinline__ void load_rows_c2r(const S* spec, C2<T>* z, long row0, long rows_total) {
  constexpr int RS = N2 + N2 / 16;
  constexpr int H = N2 / 2;
  for (int v = threadIdx.x; v < ROWS * H * 3; v += NTB) {
    const int rr = v / (H * 3), rem = v % (H * 3);
    const int k = rem / 3, q = rem % 3;
    const long row = row0 + rr;
    C2<T> a = {0, 0}, b = {0, 0};
    if (row < rows_total) {
      const S* s = spec + spec_at(row, k, 2 * q, rows_total, kchunk(H));
      a = sload<T>(s);
      b = sload<T>(s + 1);
    }
    C2<T>* zr = z + (rr * 3 + q) * RS;
    if (k == 0) {
      zr[padx<true>(0)] = C2<T>{a.x, b.x};
      zr[padx<true>(H)] = C2<T>{0, 0};
    } else {
      zr[padx<true>(k)] = C2<T>{a.x - b.y, a.y + b.x};
      zr[padx<true>(N2 - k)] = C2<T>{a.x + b.y, b.x - a.y};
    }
  }
}

template <typename T, int N2, bool ISO, int ROWS = x_rows<T>(N2), int NTB = NT, typename S = C2<T>, int PLAN = 0>
__global__ __launch_bounds__(NTB) void k_xfwd(const Desc* __restrict__ descs, int mode, long rows_total,
                                              long nvox) {
  constexpr int RS = N2 + N2 / 16;
  constexpr int H = N2 / 2;
  __shared__ C2<T> z[ROWS * 3 * RS];
  __shared__ C2<T> tw[N2];
  const Desc& d = descs[blockIdx.y];
  if (!d.st->active) return;
  build_twiddles<T, N2, NTB>(tw);
  const long row0 = (long)blockIdx.x * ROWS;
  const T* mat = mat_of<T>(d);
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  const T beta = (T)d.st->beta;
  const T ts = d.h16 ? (T)(d.tau_scale / d.st->dscale) : T(1);   // binary16 spectrum scale
  const bool first = d.st->first != 0;
  // correction fused into the FP64 residual pass (the three-term inner CG
  // leaves none after 0 iterations)
  const float* dl = (d.delta_gate && d.st2->iters == 0) ? nullptr : d.delta;

  for (int v = threadIdx.x; v < ROWS * N2; v += NTB) {
    const int rr = v / N2, i2 = v % N2;
    const long row = row0 + rr;
    T tau[6] = {0, 0, 0, 0, 0, 0};
    if (row < rows_total) {
      const long vox = row * N2 + i2;
      const int ph = d.phase[vox];
      if (mode == XF_LS) {
        T x[6] = {0, 0, 0, 0, 0, 0};
        T* xp = d.x_zero ? nullptr : (T*)d.x;
        if (xp) {
#pragma unroll
          for (int c = 0; c < 6; ++c) x[c] = xp[c * nvox + vox];
          if (dl) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
              x[c] += (T)dl[c * nvox + vox];
              xp[c * nvox + vox] = x[c];
            }
          }
        }
        T pr[6];
        if (d.P) {
#pragma unroll
          for (int c = 0; c < 6; ++c) pr[c] = (T)d.P[c * nvox + vox];
        }
        if (!d.P) {
          T e[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) e[c] = (T)d.E[c];
          apply_mat<T, ISO>(mat, ph, false, e, pr);
        }
        T dx[6];
        apply_mat<T, ISO>(mat, ph, true, x, dx);
#pragma unroll
        for (int c = 0; c < 6; ++c) tau[c] = pr[c] + dx[c];
        acc0 += frob_acc(pr, pr);
      } else if (mode == XF_MATVEC) {
        const T* vp = (const T*)d.x;
        T x[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) x[c] = vp[c * nvox + vox];
        apply_mat<T, ISO>(mat, ph, true, x, tau);
      } else if (mode == XF_CG) {
        const T* rp = (const T*)d.r;
        T* pp = (T*)d.p;
        T p[6], po[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          p[c] = rp[c * nvox + vox];
          po[c] = first ? T(0) : pp[c * nvox + vox];
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          if (!first) p[c] += beta * po[c];
          pp[c * nvox + vox] = p[c];
        }
        apply_mat<T, ISO>(mat, ph, true, p, tau);
        T cp[6];
        apply_mat<T, ISO>(mat, ph, false, p, cp);
        acc0 += frob_acc(p, cp);
      } else if (mode == XF_R3) {
        // start of the three-term CG: tau = (C - C0) r_0 and the sums
        // <r, r>_C0, <r, C r> (= <r, A r>_C0 on compatible r) and ||r||^2
        // (binary16 spectrum: tau carries the factor that keeps the transforms
        // in range, with the right-hand side's RMS divided out)
        const T* rp = (const T*)rslot(d, d.st->iters);
        T r[6], cr[6];
        double rd[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          r[c] = rp[c * nvox + vox];
          rd[c] = (double)r[c];
        }
        apply_mat<T, ISO>(mat, ph, true, r, tau);
        apply_mat<T, ISO>(mat, ph, false, r, cr);
        if (d.h16) {
#pragma unroll
          for (int c = 0; c < 6; ++c) tau[c] *= ts;
        }
        acc0 += c0_ip(d.lam0, d.mu0, rd, rd);
        acc1 += frob_acc(r, cr);
        acc2 += rd[0] * rd[0] + rd[1] * rd[1] + rd[2] * rd[2] + 2.0 * (rd[3] * rd[3] + rd[4] * rd[4] + rd[5] * rd[5]);
      } else if (mode == XF_BI1) {
        // BiCGSTAB, first pass of an iteration.  First iteration: p = r^ = r_0.
        // Later: the previous iteration's x += alpha p + omega s and r = s - omega t,
        // then p = r + beta (p - omega v).  tau = (C - C0) p.
        T* rp = (T*)d.r;
        T* pp = (T*)d.p;
        T p[6];
        if (first) {
          T* rh = (T*)d.rh;
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            const T rv = rp[c * nvox + vox];
            rh[c * nvox + vox] = rv;
            pp[c * nvox + vox] = rv;
            p[c] = rv;
          }
        } else {
          T* xp = (T*)d.x;
          const T* sp = (const T*)d.s;
          const T* tp = (const T*)d.t;
          const T* vp = (const T*)d.v;
          const T al = (T)d.st->alpha, om = (T)d.st->omega;
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            const long i = c * nvox + vox;
            const T sv = sp[i], po = pp[i];
            xp[i] += al * po + om * sv;
            const T rv = sv - om * tp[i];
            rp[i] = rv;
            p[c] = rv + beta * (po - om * vp[i]);
            pp[i] = p[c];
          }
        }
        apply_mat<T, ISO>(mat, ph, true, p, tau);
      } else if (mode == XF_BI2) {
        // BiCGSTAB, second pass: s = r - alpha v, tau = (C - C0) s
        const T* rp = (const T*)d.r;
        const T* vp = (const T*)d.v;
        T* sp = (T*)d.s;
        const T al = (T)d.st->alpha;
        T sv[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          sv[c] = rp[c * nvox + vox] - al * vp[c * nvox + vox];
          sp[c * nvox + vox] = sv[c];
        }
        apply_mat<T, ISO>(mat, ph, true, sv, tau);
      } else if (mode == XF_C0) {
        // tau = C0 : r for the projection -Gamma0 * C0 r (r is the FP64 residual)
        const double* vp = (const double*)d.r;
        T v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = (T)vp[c * nvox + vox];
        const T tr = (T)d.lam0 * (v[0] + v[1] + v[2]);
#pragma unroll
        for (int c = 0; c < 6; ++c) tau[c] = T(2) * (T)d.mu0 * v[c] + (c < 3 ? tr : T(0));
      } else {  // XF_COPY
        const double* ip = (const double*)d.io;
#pragma unroll
        for (int c = 0; c < 6; ++c)
          if (c < d.nc) tau[c] = (T)ip[c * nvox + vox];
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) z[(rr * 3 + q) * RS + padx<true>(i2)] = C2<T>{tau[2 * q], tau[2 * q + 1]};
  }
  __syncthreads();
  lds_fft<T, N2, ROWS * 3, NTB, 1, RS, false, true, -1, 1, PLAN>(z, tw);

  store_rows_r2c<T, N2, ROWS, NTB, S>((S*)d.spec, z, row0, rows_total);
  double sums[3] = {acc0, acc1, acc2};
  block_sums<3, NTB>(sums, d.part_f + blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// x-pass, inverse: complex-to-real FFT along axis 2 + update + reductions.
// ---------------------------------------------------------------------------
template <typename T, int N2, bool ISO, int ROWS = xi_rows<T>(N2), int NTB = NT, int PLAN = 0>
__global__ __launch_bounds__(NTB) void k_xinv(const Desc* __restrict__ descs, int mode, long rows_total, long nvox) {
  constexpr int RS = N2 + N2 / 16;
  constexpr int H = N2 / 2;
  __shared__ C2<T> z[ROWS * 3 * RS];
  __shared__ C2<T> tw[N2];
  const Desc& d = descs[blockIdx.y];
  if (!d.st->active) return;
  build_twiddles<T, N2, NTB>(tw);
  const long row0 = (long)blockIdx.x * ROWS;
  load_rows_c2r<T, N2, ROWS, NTB>((const C2<T>*)d.spec, z, row0, rows_total);
  __syncthreads();
  lds_fft<T, N2, ROWS * 3, NTB, 1, RS, false, true, +1, 1, PLAN>(z, tw);

  const T alpha = (T)d.st->alpha;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0, acc4 = 0.0;
  for (int v = threadIdx.x; v < ROWS * N2; v += NTB) {
    const int rr = v / N2, i2 = v % N2;
    const long row = row0 + rr;
    if (row >= rows_total) continue;
    const long vox = row * N2 + i2;
    T eta[6];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const C2<T> w = z[(rr * 3 + q) * RS + padx<true>(i2)];
      eta[2 * q] = w.x;
      eta[2 * q + 1] = w.y;
    }
    if (mode == XI_STORE || mode == XI_ACCUM) {
      double* op = (double*)d.out;
      const int nco = d.nc_out ? d.nc_out : d.nc;
      double o[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = (mode == XI_ACCUM && c < nco) ? op[c * nvox + vox] : 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (c < nco) op[c * nvox + vox] = o[c] + (double)eta[c];
    } else if (mode == XI_BS) {
      T* xp = (T*)d.x;
      T df[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) df[c] = eta[c] - xp[c * nvox + vox];
#pragma unroll
      for (int c = 0; c < 6; ++c) xp[c * nvox + vox] = eta[c];
      acc0 += frob_acc(df, df);
    } else if (mode == XI_RESID) {
      const T* xp = (const T*)d.x;
      double r[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) r[c] = (double)eta[c] - (d.x_zero ? 0.0 : (double)xp[c * nvox + vox]);
      if (d.r_f32) {
        float* rp = (float*)d.r;
#pragma unroll
        for (int c = 0; c < 6; ++c) rp[c * nvox + vox] = (float)r[c];
      } else {
        T* rp = (T*)d.r;
#pragma unroll
        for (int c = 0; c < 6; ++c) rp[c * nvox + vox] = (T)r[c];
      }
      acc0 += r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + 2.0 * (r[3] * r[3] + r[4] * r[4] + r[5] * r[5]);
      acc1 += c0_ip(d.lam0, d.mu0, r, r);
    } else if (mode == XI_BS_INNER) {
      T* xp = (T*)d.x;
      const T* rp = (const T*)d.r;
      T df[6], nv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        nv[c] = rp[c * nvox + vox] + eta[c];
        df[c] = nv[c] - xp[c * nvox + vox];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) xp[c * nvox + vox] = nv[c];
      acc0 += frob_acc(df, df);
    } else if (mode == XI_PROJ) {
      // eta = -P r.  Compatible part r_c = -eta goes to the FP32 inner right-hand
      // side; the rest, r - r_c = -(incompatible part of x), is applied to x.
      // x and r are FP64 in every instantiation (the projection itself may run
      // in FP32: it needs accuracy relative to r only).
      double* xp = (double*)d.x;
      const double* rp = (const double*)d.r;
      float* op = (float*)d.out;
      double rc[6], xv[6], rv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        xv[c] = xp[c * nvox + vox];
        rv[c] = rp[c * nvox + vox];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        rc[c] = -(double)eta[c];
        xp[c * nvox + vox] = xv[c] + (rv[c] - rc[c]);
        op[c * nvox + vox] = (float)rc[c];
      }
      acc0 += rc[0] * rc[0] + rc[1] * rc[1] + rc[2] * rc[2] + 2.0 * (rc[3] * rc[3] + rc[4] * rc[4] + rc[5] * rc[5]);
      acc1 += c0_ip(d.lam0, d.mu0, rc, rc);
    } else if (mode == XI_BI1) {
      // BiCGSTAB: v = A p = p - eta; <r^, v>
      const T* pp = (const T*)d.p;
      const T* rh = (const T*)d.rh;
      T* vp = (T*)d.v;
      T v[6], h[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        v[c] = pp[c * nvox + vox] - eta[c];
        h[c] = rh[c * nvox + vox];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) vp[c * nvox + vox] = v[c];
      acc0 += frob_d(h, v);
    } else if (mode == XI_BI2) {
      // BiCGSTAB: t = A s = s - eta; <t,s>, <t,t>, <r^,s>, <r^,t>, <s,s>
      const T* sp = (const T*)d.s;
      const T* rh = (const T*)d.rh;
      T* tp = (T*)d.t;
      T sv[6], tv[6], h[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        sv[c] = sp[c * nvox + vox];
        h[c] = rh[c * nvox + vox];
        tv[c] = sv[c] - eta[c];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) tp[c * nvox + vox] = tv[c];
      acc0 += frob_d(tv, sv);
      acc1 += frob_d(tv, tv);
      acc2 += frob_d(h, sv);
      acc3 += frob_d(h, tv);
      acc4 += frob_d(sv, sv);
    } else {  // XI_CG: q = p - eta; x += alpha p; r -= alpha q
      T* xp = (T*)d.x;
      T* rp = (T*)d.r;
      const T* pp = (const T*)d.p;
      double r[6];
      T pv[6], xv[6], rv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        pv[c] = pp[c * nvox + vox];
        xv[c] = xp[c * nvox + vox];
        rv[c] = rp[c * nvox + vox];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const T qv = pv[c] - eta[c];
        xp[c * nvox + vox] = xv[c] + alpha * pv[c];
        const T rn = rv[c] - alpha * qv;
        rp[c * nvox + vox] = rn;
        r[c] = (double)rn;
      }
      acc0 += c0_ip(d.lam0, d.mu0, r, r);
      acc1 += r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + 2.0 * (r[3] * r[3] + r[4] * r[4] + r[5] * r[5]);
    }
  }
  if (mode == XI_BI2) {
    double sums[5] = {acc0, acc1, acc2, acc3, acc4};
    block_sums<5, NTB>(sums, d.part_i + blockIdx.x, gridDim.x);
  } else {
    double sums[2] = {acc0, acc1};
    block_sums<2, NTB>(sums, d.part_i + blockIdx.x, gridDim.x);
  }
}

// ---------------------------------------------------------------------------
// Three-term CG iteration fused into one x-pass: inverse FFT of eta_k =
// -Gamma0 * (C - C0) r_k, the recurrences
//   w = A r_k = r_k - eta_k
//   r_{k+1} = omega_k (r_k - gamma_k w) + (1 - omega_k) r_{k-1}
//   x_{k+1} = omega_k (x_k + gamma_k r_k) + (1 - omega_k) x_{k-1}
// (gamma = <r,r>_C0 / <r,Ar>_C0, omega from the previous scalars; the first
// step has omega = 1; x_0 = 0 is never stored), the sums of r_{k+1} and the
// forward FFT of (C - C0) r_{k+1}, written back over the block's own spectrum
// rows.  r_k sits in slot k mod 2.  The x recurrence is applied two steps at a
// time: the odd iteration k forms x_k (from x_{k-1}, x_{k-2}, r_{k-1} and the
// previous scalars) and x_{k+1} from the same data plus r_k, the two residuals
// it reads anyway, so x is read and written on every other iteration only
// (the pair x_{k+1}, x_k overwrites x_{k-1}, x_{k-2} in slots x, x1).  A solve
// that stops after an even iteration forms its last x in k_cg3_finish.
// ---------------------------------------------------------------------------
// Row block b of nblk (its partial sums go to slot k at part_i + k nblk + b);
// z: ROWS * 3 * (N2 + N2/16) LDS elements, tw: N2.
template <typename T, int N2, bool ISO, int ROWS, int NTB, typename S, int PLAN>
__device__ __forceinline__ void xcg3_tile(const Desc& d, int b, int nblk, long rows_total, long nvox, C2<T>* z,
                                          C2<T>* tw) {
  constexpr int RS = N2 + N2 / 16;
  build_twiddles<T, N2, NTB>(tw);
  const long row0 = (long)b * ROWS;
  // binary16 inner solve: eta comes from the FP32 copy, tau goes out in binary16
  constexpr bool FULL = std::is_same<S, C2<T>>::value;
  S* spec = (S*)d.spec;
  load_rows_c2r<T, N2, ROWS, NTB>((const C2<T>*)(FULL ? d.spec : d.spec2), z, row0, rows_total);
  __syncthreads();
  lds_fft<T, N2, ROWS * 3, NTB, 1, RS, false, true, +1, 1, PLAN>(z, tw);

  const int it = d.st->iters;
  const bool first = d.st->first != 0;
  const bool xstep = (it & 1) != 0;   // this iteration forms x_k and x_{k+1}
  const T gam = (T)d.st->alpha;
  const T om = first ? T(1) : (T)d.st->beta;
  const T gp = (T)d.st->alpha_prev;   // gamma_{k-1}
  const T op = (T)d.st->beta_prev;    // omega_{k-1} (1 at k = 1)
  const T* rc = (const T*)rslot(d, it);        // r_k
  const T* rpv = (const T*)rslot(d, it + 1);   // r_{k-1}, overwritten by r_{k+1}
  T* ro = (T*)rslot(d, it + 1);
  T* xn = (T*)d.x;    // x_{k-1} in, x_{k+1} out (odd k)
  T* xo = (T*)d.x1;   // x_{k-2} in, x_k out
  const T* mat = mat_of<T>(d);
  const T ts = d.h16 ? (T)(d.tau_scale / d.st->dscale) : T(1);   // binary16 spectrum scale
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  for (int v = threadIdx.x; v < ROWS * N2; v += NTB) {
    const int rr = v / N2, i2 = v % N2;
    const long row = row0 + rr;
    T tau[6] = {0, 0, 0, 0, 0, 0};
    if (row < rows_total) {
      const long vox = row * N2 + i2;
      const int ph = d.phase[vox];
      // every load of the voxel is issued before the first store (the output
      // slots may alias the inputs as far as the compiler knows)
      // (the iterates are streamed: each is read once per iteration, long after
      // it was written, so the accesses carry the non-temporal hint)
      T rk[6], rp[6], xa[6], xb[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        rk[c] = __builtin_nontemporal_load(rc + c * nvox + vox);
        rp[c] = first ? T(0) : __builtin_nontemporal_load(rpv + c * nvox + vox);
        // x_0 = 0 is never stored: the pair is read from the third iteration on
        xa[c] = (xstep && it > 1) ? __builtin_nontemporal_load(xn + c * nvox + vox) : T(0);
        xb[c] = (xstep && it > 1) ? __builtin_nontemporal_load(xo + c * nvox + vox) : T(0);
      }
      T rn[6];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const C2<T> e = z[(rr * 3 + q) * RS + padx<true>(i2)];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int c = 2 * q + h;
          const T eta = h ? e.y : e.x;
          const T r = rk[c];
          const T w = r - eta;
          const T rv = first ? r - gam * w : om * (r - gam * w) + (T(1) - om) * rp[c];
          __builtin_nontemporal_store(rv, ro + c * nvox + vox);
          if (xstep) {
            const T xk = op * (xa[c] + gp * rp[c]) + (T(1) - op) * xb[c];
            const T x1 = om * (xk + gam * r) + (T(1) - om) * xa[c];
            __builtin_nontemporal_store(x1, xn + c * nvox + vox);
            __builtin_nontemporal_store(xk, xo + c * nvox + vox);
          }
          rn[c] = rv;
        }
      }
      T cr[6];
      double rd[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) rd[c] = (double)rn[c];
      apply_mat<T, ISO>(mat, ph, true, rn, tau);
      apply_mat<T, ISO>(mat, ph, false, rn, cr);
      acc0 += c0_ip(d.lam0, d.mu0, rd, rd);
      acc1 += frob_acc(rn, cr);
      acc2 += rd[0] * rd[0] + rd[1] * rd[1] + rd[2] * rd[2] + 2.0 * (rd[3] * rd[3] + rd[4] * rd[4] + rd[5] * rd[5]);
      if (d.h16) {
#pragma unroll
        for (int c = 0; c < 6; ++c) tau[c] *= ts;
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) z[(rr * 3 + q) * RS + padx<true>(i2)] = C2<T>{tau[2 * q], tau[2 * q + 1]};
  }
  __syncthreads();
  lds_fft<T, N2, ROWS * 3, NTB, 1, RS, false, true, -1, 1, PLAN>(z, tw);
  store_rows_r2c<T, N2, ROWS, NTB, S>(spec, z, row0, rows_total);
  double sums[3] = {acc0, acc1, acc2};
  block_sums<3, NTB>(sums, d.part_i + b, nblk);
}

template <typename T, int N2, bool ISO, int ROWS = xi_rows<T>(N2), int NTB = NT, typename S = C2<T>, int PLAN = 0>
__global__ __launch_bounds__(NTB) void k_xcg3(const Desc* __restrict__ descs, long rows_total, long nvox) {
  __shared__ C2<T> z[ROWS * 3 * (N2 + N2 / 16)];
  __shared__ C2<T> tw[N2];
  const Desc& d = descs[blockIdx.y];
  if (!d.st->active) return;
  xcg3_tile<T, N2, ISO, ROWS, NTB, S, PLAN>(d, (int)blockIdx.x, (int)gridDim.x, rows_total, nvox, z, tw);
}

// Three-term CG: the last x of loads whose solve stopped after an even
// iteration k (their state says so).  The odd iteration k - 1 left x_k and
// x_{k-1} in the slots x and x1; x_{k+1} = omega_k (x_k + gamma_k r_k) +
// (1 - omega_k) x_{k-1} goes to x (k = 0: x_1 = gamma_0 r_0); nothing reads
// x1 after a solve, so it is left as it is.  n = 6 x voxels.  Run once per
// stopped solve (the update is not idempotent).
template <typename T>
__global__ __launch_bounds__(NT) void k_cg3_finish(const Desc* __restrict__ descs, long n) {
  const Desc& d = descs[blockIdx.y];
  const SolverState* st = d.st;
  if (st->active || !st->xpend) return;
  const int k = st->iters - 1;
  const T gam = (T)st->alpha;
  const T om = k == 0 ? T(1) : (T)st->beta;
  const T* rk = (const T*)rslot(d, k);
  T* xn = (T*)d.x;
  const T* xo = (const T*)d.x1;
  for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) {
    if (k == 0) {
      xn[i] = gam * rk[i];
    } else {
      const T xa = xn[i], xb = xo[i];
      xn[i] = om * (xa + gam * rk[i]) + (T(1) - om) * xb;
    }
  }
}

// BiCGSTAB: apply the last iteration's x += alpha p + omega s to loads that
// stopped (the next iteration's first pass would have done it).
template <typename T>
__global__ __launch_bounds__(NT) void k_bicg_finish(const Desc* __restrict__ descs, long n) {
  const Desc& d = descs[blockIdx.y];
  const SolverState* st = d.st;
  if (st->active || !st->pending) return;
  T* xp = (T*)d.x;
  const T* pp = (const T*)d.p;
  const T* sp = (const T*)d.s;
  const T al = (T)st->alpha, om = (T)st->omega;
  for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) xp[i] += al * pp[i] + om * sp[i];
}

// ---------------------------------------------------------------------------
// y-pass: complex FFT along axis 1, in place.  Block = one i0 plane, CW
// consecutive columns of the [n1][n2/2 * 6] plane.
// ---------------------------------------------------------------------------
// ncols is a multiple of 6, so an access group of 2 columns is either all
// inside or all outside the plane (groups of 4 are used only when ncols is a
// multiple of 4).
// S = H2 (binary16 storage): the forward transform is divided by N1 so that
// the stored values stay in range.
// Binary16 tile transfers, G columns per access (ncols and c0 multiples of G,
// so a group is either all inside or all outside the plane).
// Tile loads of the y-pass: all of a thread's global loads are issued before
// its first LDS write, so their latencies overlap.
template <typename T, int N1, int CW, int NTB, int G, typename S>
__device__ __forceinline__ void y_tile_load(const S* base, int ncols, int c0, C2<T>* buf) {
  constexpr int NA = N1 * CW / G, NL = (NA + NTB - 1) / NTB;
  C2<T> a[NL][G];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int v = threadIdx.x + k * NTB;
    const int i1 = v / (CW / G), col = (v % (CW / G)) * G;
    if ((NA % NTB == 0 || v < NA) && c0 + col < ncols) {
      if constexpr (std::is_same<S, H2>::value) hload_g<T, G>(base + (long)i1 * ncols + col, a[k]);
      else load_v<T, G>(base + (long)i1 * ncols + col, a[k]);
    } else {
#pragma unroll
      for (int q = 0; q < G; ++q) a[k][q] = C2<T>{0, 0};
    }
  }
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int v = threadIdx.x + k * NTB;
    const int i1 = v / (CW / G), col = (v % (CW / G)) * G;
    if (NA % NTB == 0 || v < NA) {
#pragma unroll
      for (int q = 0; q < G; ++q) buf[i1 * CW + col + q] = a[k][q];
    }
  }
}
template <typename T, int N1, int CW, int NTB, int G>
__device__ __forceinline__ void y_h2_store(H2* base, int ncols, int c0, const C2<T>* buf, T scale) {
  for (int v = threadIdx.x; v < N1 * CW / G; v += NTB) {
    const int i1 = v / (CW / G), col = (v % (CW / G)) * G;
    if (c0 + col < ncols) {
      C2<T> a[G];
#pragma unroll
      for (int q = 0; q < G; ++q) a[q] = buf[i1 * CW + col + q] * scale;
      hstore_g<T, G>(base + (long)i1 * ncols + col, a);
    }
  }
}

template <typename T, int N1, int CW, int NTB, int DIR, int V, typename S, int PLAN>
__device__ __forceinline__ void ypass_body(S* base, int ncols, int c0, C2<T>* buf, const C2<T>* tw) {
  constexpr bool FULL = std::is_same<S, C2<T>>::value;
  static_assert(FULL || V == 1, "binary16 storage keeps one sequence per LDS slot");
  // binary16: up to 4 columns (16 bytes) per access when the plane width allows
  constexpr int G = CW % 4 == 0 ? 4 : CW % 2 == 0 ? 2 : 1;
  const bool wide = ncols % G == 0;
  // FP32: two columns (16 bytes) per access (ncols = 6 kc is even)
  constexpr int GF = (sizeof(T) == 4 && CW % 2 == 0) ? 2 : 1;
  if constexpr (FULL) {
    y_tile_load<T, N1, CW, NTB, GF>(base, ncols, c0, buf);
  } else {
    if (wide) y_tile_load<T, N1, CW, NTB, G>(base, ncols, c0, buf);
    else y_tile_load<T, N1, CW, NTB, 1>(base, ncols, c0, buf);
  }
  __syncthreads();
  lds_fft<T, N1, CW, NTB, CW, 1, true, false, DIR, V, PLAN>(buf, tw);
  if constexpr (FULL) {
    for (int v = threadIdx.x; v < N1 * CW / GF; v += NTB) {
      const int i1 = v / (CW / GF), col = (v % (CW / GF)) * GF;
      if (c0 + col < ncols) {
        C2<T> a[GF];
#pragma unroll
        for (int q = 0; q < GF; ++q) a[q] = buf[i1 * CW + col + q];
        store_v<T, GF>(base + (long)i1 * ncols + col, a);
      }
    }
  } else {
    // the forward transform is divided by N1 so that the stored values stay in range
    const T sc = DIR < 0 ? T(1) / T(N1) : T(1);
    if (wide) y_h2_store<T, N1, CW, NTB, G>(base, ncols, c0, buf, sc);
    else y_h2_store<T, N1, CW, NTB, 1>(base, ncols, c0, buf, sc);
  }
}

// Tile bid (plane i0 = bid / ntiles, columns from (bid % ntiles) CW) of one
// load; buf: N1 * CW LDS elements (16-byte aligned), tw: N1.
template <typename T, int N1, int CW, int NTB, int V, typename S, int PLAN>
__device__ __forceinline__ void ypass_tile(const Desc& d, int bid, int dir, int ncols, int ntiles, C2<T>* buf,
                                           C2<T>* tw) {
  build_twiddles<T, N1, NTB>(tw);
  const long i0 = bid / ntiles;
  const int c0 = (bid % ntiles) * CW;
  // binary16 inner solve (spec2 set only in its descriptors): the inverse
  // y-transform runs in FP32 on the copy the spectral operator wrote
  const bool alt = std::is_same<S, C2<T>>::value && d.spec2 != nullptr && dir > 0;
  S* base = (S*)(alt ? d.spec2 : d.spec) + i0 * N1 * (long)ncols + c0;
  if (dir < 0) ypass_body<T, N1, CW, NTB, -1, V, S, PLAN>(base, ncols, c0, buf, tw);
  else ypass_body<T, N1, CW, NTB, +1, V, S, PLAN>(base, ncols, c0, buf, tw);
}

template <typename T, int N1, int CW = y_cols<T>(N1), int NTB = y_threads<T>(N1), bool REMAP = true,
          int V = vec_width<T>(), typename S = C2<T>, int PLAN = 0>
__global__ __launch_bounds__(NTB) void k_ypass(const Desc* __restrict__ descs, int dir, int ncols, int ntiles) {
  __shared__ __attribute__((aligned(16))) C2<T> buf[N1 * CW];
  __shared__ C2<T> tw[N1];
  const Desc& d = descs[blockIdx.y];
  if (!d.st->active) return;
  const int bid = REMAP ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  ypass_tile<T, N1, CW, NTB, V, S, PLAN>(d, bid, dir, ncols, ntiles, buf, tw);
}

// ---------------------------------------------------------------------------
// z-pass: forward FFT along axis 0, spectral operator, inverse FFT.
// Block = TK consecutive (i1, k2) columns x 6 components x all i0.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void spectral_op(int op, T (&in)[6][2], T (&out)[6][2], T k0, T k1, T k2, double lam0,
                                            double mu0, T scale) {
  const T kk = k0 * k0 + k1 * k1 + k2 * k2;
  const T inv = T(1) / sqrt(kk);
  const T n[3] = {k0 * inv, k1 * inv, k2 * inv};
  if (op == OP_GAMMA) {
    // eta_hat = -[ (n x v + v x n) / (2 mu0) - c2 (n.v) n x n ],  v = tau_hat n
    const T c2 = (T)((lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)));
    const T h = (T)(0.5 / mu0);
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const T t0 = in[0][ri], t1 = in[1][ri], t2 = in[2][ri], t3 = in[3][ri], t4 = in[4][ri], t5 = in[5][ri];
      const T v0 = t0 * n[0] + t5 * n[1] + t4 * n[2];
      const T v1 = t5 * n[0] + t1 * n[1] + t3 * n[2];
      const T v2 = t4 * n[0] + t3 * n[1] + t2 * n[2];
      const T s = (n[0] * v0 + n[1] * v1 + n[2] * v2) * c2;
      out[0][ri] = -scale * (T(2) * h * n[0] * v0 - s * n[0] * n[0]);
      out[1][ri] = -scale * (T(2) * h * n[1] * v1 - s * n[1] * n[1]);
      out[2][ri] = -scale * (T(2) * h * n[2] * v2 - s * n[2] * n[2]);
      out[3][ri] = -scale * (h * (n[1] * v2 + n[2] * v1) - s * n[1] * n[2]);
      out[4][ri] = -scale * (h * (n[0] * v2 + n[2] * v0) - s * n[0] * n[2]);
      out[5][ri] = -scale * (h * (n[0] * v1 + n[1] * v0) - s * n[0] * n[1]);
    }
  } else if (op == OP_THETA) {
    // theta_hat_ij = (i/|xi|) [ n_i n_j (g.n) - (g_i n_j + n_i g_j) ],  |xi| = 2 pi |k|
    const T f = scale * inv * (T)(0.5 / 3.14159265358979323846);
    T w[6][2];
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const T g0 = in[0][ri], g1 = in[1][ri], g2 = in[2][ri];
      const T gn = g0 * n[0] + g1 * n[1] + g2 * n[2];
      w[0][ri] = n[0] * n[0] * gn - T(2) * g0 * n[0];
      w[1][ri] = n[1] * n[1] * gn - T(2) * g1 * n[1];
      w[2][ri] = n[2] * n[2] * gn - T(2) * g2 * n[2];
      w[3][ri] = n[1] * n[2] * gn - (g1 * n[2] + n[1] * g2);
      w[4][ri] = n[0] * n[2] * gn - (g0 * n[2] + n[0] * g2);
      w[5][ri] = n[0] * n[1] * gn - (g0 * n[1] + n[0] * g1);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {  // multiply by i f
      out[c][0] = -f * w[c][1];
      out[c][1] = f * w[c][0];
    }
  } else {  // OP_DISP: u_hat = (-i/|xi|) [ 2 eps_hat n - n (n . eps_hat n) ]
    const T f = scale * inv * (T)(0.5 / 3.14159265358979323846);
    T w[3][2];
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const T t0 = in[0][ri], t1 = in[1][ri], t2 = in[2][ri], t3 = in[3][ri], t4 = in[4][ri], t5 = in[5][ri];
      const T v0 = t0 * n[0] + t5 * n[1] + t4 * n[2];
      const T v1 = t5 * n[0] + t1 * n[1] + t3 * n[2];
      const T v2 = t4 * n[0] + t3 * n[1] + t2 * n[2];
      const T s = n[0] * v0 + n[1] * v1 + n[2] * v2;
      w[0][ri] = T(2) * v0 - n[0] * s;
      w[1][ri] = T(2) * v1 - n[1] * s;
      w[2][ri] = T(2) * v2 - n[2] * s;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {  // multiply by -i f
      out[c][0] = f * w[c][1];
      out[c][1] = -f * w[c][0];
    }
    out[3][0] = out[3][1] = out[4][0] = out[4][1] = out[5][0] = out[5][1] = T(0);
  }
}

// Tile bid (chunk bid / bpc, columns from (bid % bpc) TK) of one load; buf:
// N0 * 6 TK LDS elements (16-byte aligned), tw: N0.
template <typename T, int N0, int TK, int NTB, int V, typename S, int PLAN>
__device__ __forceinline__ void zpass_tile(const Desc& d, int bid, int op, int n1, int h, double scale, C2<T>* buf,
                                           C2<T>* tw) {
  constexpr int W = TK * 6;
  build_twiddles<T, N0, NTB>(tw);
  // columns (i1, k2 % kc) of one k2-chunk form a [N0][M][6] sub-array
  const int kc = kchunk(h);
  const long M = (long)n1 * kc;
  const int bpc = (int)((M + TK - 1) / TK);            // blocks per chunk
  const int chunk = bid / bpc;
  const long m0 = (long)(bid % bpc) * TK;
  constexpr bool FULL = std::is_same<S, C2<T>>::value;
  // global accesses move GZ adjacent components (16 bytes in FP32, 8 in
  // binary16); W is even and so is every column's offset, so a group never
  // straddles a column
  constexpr int GZ = sizeof(T) == 4 ? 2 : 1;
  S* spec = (S*)d.spec + (long)chunk * N0 * M * 6;
  // binary16 input; the output (after the spectral operator) goes to the FP32 copy
  C2<T>* dst = (C2<T>*)(FULL ? d.spec : d.spec2) + (long)chunk * N0 * M * 6;
  // binary16 storage: the spectral operator also restores the scale of the
  // forward transforms (the descriptor's factor times the right-hand side's
  // RMS replaces 1/N)
  const T sc = FULL ? (T)scale : (T)(d.op_scale * d.st->dscale);
  // all of a thread's loads are issued before the first LDS write, so their
  // latencies overlap (the tile's rows are far apart in memory)
  constexpr int NA = N0 * W / GZ, NL = (NA + NTB - 1) / NTB;
  {
    C2<T> a[NL][GZ];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int v = threadIdx.x + k * NTB;
      const int i0 = v / (W / GZ), w = (v % (W / GZ)) * GZ;
      if ((NA % NTB == 0 || v < NA) && m0 + w / 6 < M) {
        if constexpr (FULL) load_v<T, GZ>(spec + ((long)i0 * M + m0) * 6 + w, a[k]);
        else hload_g<T, GZ>(spec + ((long)i0 * M + m0) * 6 + w, a[k]);
      } else {
#pragma unroll
        for (int q = 0; q < GZ; ++q) a[k][q] = C2<T>{0, 0};
      }
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int v = threadIdx.x + k * NTB;
      const int i0 = v / (W / GZ), w = (v % (W / GZ)) * GZ;
      if (NA % NTB == 0 || v < NA) {
#pragma unroll
        for (int q = 0; q < GZ; ++q) buf[i0 * W + w + q] = a[k][q];
      }
    }
  }
  __syncthreads();
  if constexpr (N0 > 1) lds_fft<T, N0, W, NTB, W, 1, true, false, -1, V, PLAN>(buf, tw);
  for (int v = threadIdx.x; v < N0 * TK; v += NTB) {
    const int k0 = v / TK, col = v % TK;
    const long m = m0 + col;
    if (m >= M) continue;
    const int k1 = (int)(m / kc), k2 = chunk * kc + (int)(m % kc);
    const bool nyq = ((N0 % 2 == 0) && k0 == N0 / 2) || ((n1 % 2 == 0) && k1 == n1 / 2);
    const int k0s = k0 < (N0 + 1) / 2 ? k0 : k0 - N0;
    const int k1s = k1 < (n1 + 1) / 2 ? k1 : k1 - n1;
    C2<T>* e = buf + k0 * W + col * 6;
    T in[6][2], out[6][2];
#pragma unroll
    for (int c = 0; c < 6; c += V) {
      C2<T> a[V];
      load_v<T, V>(e + c, a);
#pragma unroll
      for (int q = 0; q < V; ++q) {
        in[c + q][0] = a[q].x;
        in[c + q][1] = a[q].y;
      }
    }
    if (nyq || (k0s == 0 && k1s == 0 && k2 == 0)) {
#pragma unroll
      for (int c = 0; c < 6; ++c) out[c][0] = out[c][1] = T(0);
    } else {
      spectral_op<T>(op, in, out, (T)k0s, (T)k1s, (T)k2, d.lam0, d.mu0, sc);
    }
#pragma unroll
    for (int c = 0; c < 6; c += V) {
      C2<T> a[V];
#pragma unroll
      for (int q = 0; q < V; ++q) a[q] = C2<T>{out[c + q][0], out[c + q][1]};
      store_v<T, V>(e + c, a);
    }
  }
  __syncthreads();
  if constexpr (N0 > 1) lds_fft<T, N0, W, NTB, W, 1, true, false, +1, V, PLAN>(buf, tw);
  for (int v = threadIdx.x; v < N0 * W / GZ; v += NTB) {
    const int i0 = v / (W / GZ), w = (v % (W / GZ)) * GZ;
    if (m0 + w / 6 < M) {
      C2<T> a[GZ];
#pragma unroll
      for (int q = 0; q < GZ; ++q) a[q] = buf[i0 * W + w + q];
      if constexpr (FULL || TK % 4 != 0) {
        store_v<T, GZ>(dst + ((long)i0 * M + m0) * 6 + w, a);
      } else {
        // the FP32 copy after the operator goes to its own buffer: streamed
        // with the non-temporal hint, which pays only when every row segment
        // (48 TK bytes) covers whole 64-byte chunks
        static_assert(GZ == 2, "binary16 input implies FP32 pairs");
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 o = {a[0].x, a[0].y, a[1].x, a[1].y};
        __builtin_nontemporal_store(o, (f4*)(dst + ((long)i0 * M + m0) * 6 + w));
      }
    }
  }
}

template <typename T, int N0, int TK = z_cols<T>(N0), int NTB = NT, bool REMAP = true, int V = vec_width<T>(),
          typename S = C2<T>, int PLAN = 0>
__global__ __launch_bounds__(NTB) void k_zpass(const Desc* __restrict__ descs, int op, int n1, int h, double scale) {
  __shared__ __attribute__((aligned(16))) C2<T> buf[N0 * TK * 6];
  __shared__ C2<T> tw[N0];
  const Desc& d = descs[blockIdx.y];
  if (!d.st->active) return;
  const int bid = REMAP ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  zpass_tile<T, N0, TK, NTB, V, S, PLAN>(d, bid, op, n1, h, scale, buf, tw);
}

// ---------------------------------------------------------------------------
// Multi-size launches of the FP32 inner iteration: one launch per pass
// covers loads of grids of different sizes (axis lengths from
// FFTH_MULTI_SIZES).  Each load's descriptor carries its grid (n); the
// launch's blocks are the tiles of all its loads, listed by a segment table
// (MultiSegs) of consecutive loads of one grid, each tile with the default
// tile shape of its lengths (variant 0, radix plan 0, 256 threads: the
// arithmetic of the per-size kernels with their default tiles, bit for bit).
// LDS is sized for the largest length.
// ---------------------------------------------------------------------------
#define FFTH_MULTI_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128)
constexpr int MULTI_NT = 256;
constexpr int MULTI_MAXN = 128;
constexpr int MULTI_SIZES[] = {16, 24, 32, 48, 64, 96, 128};   // the lengths of FFTH_MULTI_SIZES
constexpr bool multi_size(int n) {
  for (int m : MULTI_SIZES)
    if (m == n) return true;
  return false;
}
#define FFTH_MULTI_CHECK(N) static_assert(multi_size(N), "FFTH_MULTI_SIZES and MULTI_SIZES differ");
FFTH_MULTI_SIZES(FFTH_MULTI_CHECK)
#undef FFTH_MULTI_CHECK
#define FFTH_MULTI_COUNT(N) +1
static_assert(0 FFTH_MULTI_SIZES(FFTH_MULTI_COUNT) == sizeof(MULTI_SIZES) / sizeof(int), "FFTH_MULTI_SIZES and MULTI_SIZES differ");
#undef FFTH_MULTI_COUNT
// blocks of one load of grid n in each multi-size pass (host and device)
__host__ __device__ constexpr int multi_y_blocks(int n0, int n1, int n2) {
  const int h = n2 / 2, kc = kchunk(h), cw = y_cols<float>(n1);
  return n0 * (h / kc) * ((kc * 6 + cw - 1) / cw);
}
__host__ __device__ constexpr int multi_z_blocks(int n0, int n1, int n2) {
  const int h = n2 / 2, kc = kchunk(h), tk = z_cols<float>(n0);
  return (int)(((long)n1 * kc + tk - 1) / tk) * (h / kc);
}
__host__ __device__ constexpr int multi_x_blocks(int n0, int n1, int n2) {
  const int r = xi_rows<float>(n2);
  return (int)(((long)n0 * n1 + r - 1) / r);
}
// FP32 LDS elements of each pass at length n, and their maxima over the set
constexpr int multi_lds(int pass, int n) {
  return pass == 0 ? n * y_cols<float>(n) : pass == 1 ? n * 6 * z_cols<float>(n) : xi_rows<float>(n) * 3 * (n + n / 16);
}
constexpr int multi_lds_max(int pass) {
  int m = 0;
  for (int n : MULTI_SIZES) m = multi_lds(pass, n) > m ? multi_lds(pass, n) : m;
  return m;
}
constexpr int MULTI_LDS_Y = multi_lds_max(0), MULTI_LDS_Z = multi_lds_max(1), MULTI_LDS_X = multi_lds_max(2);

// Block of a multi-size launch: its load (descriptor index, -1 for padding)
// and that load's tile.  Each load of segment s owns bpd[s] blocks padded to
// a multiple of 8 (the XCDs; segments start at multiples of 8 too), so a
// block's XCD is its tile slot mod 8; with REMAP the tiles of every load are
// renumbered XCD-aware as the per-size y and z passes do (each XCD walks a
// contiguous run of each load's tiles), without it a load's tiles are taken
// in order as in the per-size fused pass.
template <bool REMAP> __device__ __forceinline__ int multi_block(const MultiSegs& sg, int& tile) {
  const int b = blockIdx.x;
  int s = 0;
  while (s + 1 < sg.n && b >= sg.off[s + 1]) ++s;
  const int bpd = sg.bpd[s], slots = (bpd + 7) / 8 * 8;
  const int r = b - sg.off[s], load = r / slots, t = r % slots;
  if (t >= bpd) return -1;
  tile = REMAP ? xcd_tile(t, bpd) : t;
  return sg.first[s] + load;
}
template <typename S>
__global__ __launch_bounds__(MULTI_NT) void k_ypass_multi(const Desc* __restrict__ descs, int dir, MultiSegs sg) {
  __shared__ __attribute__((aligned(16))) C2<float> buf[MULTI_LDS_Y];
  __shared__ C2<float> tw[MULTI_MAXN];
  int bid;
  const int di = multi_block<true>(sg, bid);
  if (di < 0) return;
  const Desc& d = descs[di];
  if (!d.st->active) return;
  const int kc = kchunk(d.n[2] / 2), ncols = kc * 6;
  switch (d.n[1]) {
#define FFTH_MULTI_Y(N)                                                                                   \
  case N: {                                                                                               \
    constexpr int CW = y_cols<float>(N);                                                                  \
    ypass_tile<float, N, CW, MULTI_NT, 1, S, 0>(d, bid, dir, ncols, (ncols + CW - 1) / CW, buf, tw);    \
    break;                                                                                                \
  }
    FFTH_MULTI_SIZES(FFTH_MULTI_Y)
#undef FFTH_MULTI_Y
  }
}

template <typename S>
__global__ __launch_bounds__(MULTI_NT) void k_zpass_multi(const Desc* __restrict__ descs, int op, MultiSegs sg) {
  __shared__ __attribute__((aligned(16))) C2<float> buf[MULTI_LDS_Z];
  __shared__ C2<float> tw[MULTI_MAXN];
  int bid;
  const int di = multi_block<true>(sg, bid);
  if (di < 0) return;
  const Desc& d = descs[di];
  if (!d.st->active) return;
  switch (d.n[0]) {
#define FFTH_MULTI_Z(N)                                                                                   \
  case N:                                                                                                 \
    zpass_tile<float, N, z_cols<float>(N), MULTI_NT, 1, S, 0>(d, bid, op, d.n[1], d.n[2] / 2, d.inv_nvox, buf, tw); \
    break;
    FFTH_MULTI_SIZES(FFTH_MULTI_Z)
#undef FFTH_MULTI_Z
  }
}

// The tile of the fused pass is the load's row block b, whose partial sums
// go to slot b of the load's array.
template <bool ISO, typename S>
__global__ __launch_bounds__(MULTI_NT) void k_xcg3_multi(const Desc* __restrict__ descs, MultiSegs sg) {
  __shared__ C2<float> z[MULTI_LDS_X];
  __shared__ C2<float> tw[MULTI_MAXN];
  int b;
  const int di = multi_block<false>(sg, b);
  if (di < 0) return;
  const Desc& d = descs[di];
  if (!d.st->active) return;
  const int nb = multi_x_blocks(d.n[0], d.n[1], d.n[2]);
  const long rows = (long)d.n[0] * d.n[1];
  switch (d.n[2]) {
#define FFTH_MULTI_X(N)                                                                                   \
  case N:                                                                                                 \
    xcg3_tile<float, N, ISO, xi_rows<float>(N), MULTI_NT, S, 0>(d, b, nb, rows, rows * N, z, tw);        \
    break;
    FFTH_MULTI_SIZES(FFTH_MULTI_X)
#undef FFTH_MULTI_X
  }
}

// ---------------------------------------------------------------------------
// Finalize: fixed-order sum of the block partials of one batch entry, then
// the scalar update of its iteration state.  One block per entry.
// ---------------------------------------------------------------------------
constexpr int NT_FIN = 1024;
__global__ __launch_bounds__(NT_FIN) void k_finalize(const Desc* __restrict__ descs, int op, int nblk_f, int nblk_i);

// Volume averages of sigma = P_rhs + C:x (or C:(E + x)): 6 sums per block.
template <bool ISO>
__global__ __launch_bounds__(NT) void k_mean_stress(const Desc* __restrict__ descs, long nvox);

// Order-1 pointwise right-hand side: P = C:sym(X1.G), g_i = sum_J c_J S^J_ij G_Jj.
template <bool ISO>
__global__ __launch_bounds__(NT) void k_order1_point(const Desc* __restrict__ descs, const double* __restrict__ eps0,
                                                     const double* __restrict__ x1, long nvox);

// out <- (double) x for FP32 x, n values.
__global__ void k_widen(const Desc* __restrict__ descs, long n);

// Largest phase id (validation of the problem input).
__global__ void k_phase_max(const uint16_t* __restrict__ phase, long n, int* out);

}  // namespace ffth
