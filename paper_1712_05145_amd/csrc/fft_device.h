// Device building blocks for the 3-D real FFTs of the homogenization solver:
// complex arithmetic, radix-2/3/4/5/8/16 butterflies in registers, a
// mixed-radix Stockham FFT over batches of sequences resident in LDS, and
// wave/block reductions.  gfx950 (CDNA4): 64-wide wavefronts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffth {

template <typename T> struct C2 { T x, y; };

template <typename T> __device__ __forceinline__ C2<T> mk(T a, T b) { return C2<T>{a, b}; }
template <typename T> __device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ C2<T> operator-(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ C2<T> operator*(C2<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ C2<T> conj(C2<T> a) { return {a.x, -a.y}; }
// multiply by +i (DIR>0) or -i (DIR<0)
template <int DIR, typename T> __device__ __forceinline__ C2<T> mul_i(C2<T> a) {
  return DIR > 0 ? C2<T>{-a.y, a.x} : C2<T>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Compile-time factorisation of a transform length into the radices 16, 8,
// 4, 2, 3, 5.  A radix plan is the order in which the radices are preferred:
// each stage takes the first preferred radix that divides what is left.
//   plan 0: 16, 8, 4, 2, 3, 5   (fewest stages: 256 = 16 x 16)
//   plan 1:  4, 2, 3, 5, 8, 16  (small butterflies: 256 = 4 x 4 x 4 x 4)
//   plan 2:  8, 4, 2, 3, 5, 16  (256 = 8 x 8 x 4)
// The run-time tuner times the plans (with the default tile shape) beside the
// tile shapes of every pass.
// ---------------------------------------------------------------------------
constexpr int NPLAN = 3;
constexpr int plan_radix(int plan, int i) {
  constexpr int rs[NPLAN][6] = {{16, 8, 4, 2, 3, 5}, {4, 2, 3, 5, 8, 16}, {8, 4, 2, 3, 5, 16}};
  return rs[plan][i];
}
constexpr int fac_count(int n, int plan = 0) {
  int c = 0;
  for (int i = 0; i < 6; ++i)
    while (n > 1 && n % plan_radix(plan, i) == 0) { n /= plan_radix(plan, i); ++c; }
  return n == 1 ? c : -1;
}
constexpr int fac_radix(int n, int s, int plan = 0) {
  int c = 0;
  for (int i = 0; i < 6; ++i)
    while (n > 1 && n % plan_radix(plan, i) == 0) {
      if (c == s) return plan_radix(plan, i);
      n /= plan_radix(plan, i);
      ++c;
    }
  return 1;
}
constexpr int fac_prefix(int n, int s, int plan = 0) {  // product of radices before stage s
  int p = 1;
  for (int i = 0; i < s; ++i) p *= fac_radix(n, i, plan);
  return p;
}

// ---------------------------------------------------------------------------
// Small DFTs in registers.  DIR = -1 forward (exp(-2 pi i/R)), +1 inverse.
// ---------------------------------------------------------------------------
#define FFTH_C16_1 0.92387953251128675613
#define FFTH_S16_1 0.38268343236508977173
#define FFTH_SQRT_HALF 0.70710678118654752440
#define FFTH_S3 0.86602540378443864676
#define FFTH_C5_1 0.30901699437494742410
#define FFTH_S5_1 0.95105651629515357212
#define FFTH_C5_2 (-0.80901699437494742410)
#define FFTH_S5_2 0.58778525229247312917

template <int DIR, typename T> __device__ __forceinline__ void dft2(C2<T>& a, C2<T>& b) {
  C2<T> t = a;
  a = t + b;
  b = t - b;
}

template <int DIR, typename T> __device__ __forceinline__ void dft4(C2<T>& a0, C2<T>& a1, C2<T>& a2, C2<T>& a3) {
  C2<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_i<DIR>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <int DIR, typename T> __device__ __forceinline__ void dft3(C2<T>& a0, C2<T>& a1, C2<T>& a2) {
  // X1 = a0 + w a1 + w^2 a2, w = exp(DIR 2 pi i/3) = -1/2 + DIR i sqrt(3)/2
  C2<T> s = a1 + a2, d = a1 - a2;
  C2<T> m = a0 - s * T(0.5);
  C2<T> r = mul_i<DIR>(d) * T(FFTH_S3);
  a0 = a0 + s;
  a1 = m + r;
  a2 = m - r;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft5(C2<T>& a0, C2<T>& a1, C2<T>& a2, C2<T>& a3, C2<T>& a4) {
  C2<T> s1 = a1 + a4, d1 = a1 - a4, s2 = a2 + a3, d2 = a2 - a3;
  C2<T> m1 = a0 + s1 * T(FFTH_C5_1) + s2 * T(FFTH_C5_2);
  C2<T> m2 = a0 + s1 * T(FFTH_C5_2) + s2 * T(FFTH_C5_1);
  C2<T> r1 = mul_i<DIR>(d1 * T(FFTH_S5_1) + d2 * T(FFTH_S5_2));
  C2<T> r2 = mul_i<DIR>(d1 * T(FFTH_S5_2) - d2 * T(FFTH_S5_1));
  a0 = a0 + s1 + s2;
  a1 = m1 + r1;
  a4 = m1 - r1;
  a2 = m2 + r2;
  a3 = m2 - r2;
}

// exp(DIR * 2 pi i * m / 16) for m in [0, 16)
template <int DIR, typename T> __device__ __forceinline__ C2<T> w16(int m) {
  const T c[16] = {T(1), T(FFTH_C16_1), T(FFTH_SQRT_HALF), T(FFTH_S16_1), T(0), T(-FFTH_S16_1),
                   T(-FFTH_SQRT_HALF), T(-FFTH_C16_1), T(-1), T(-FFTH_C16_1), T(-FFTH_SQRT_HALF),
                   T(-FFTH_S16_1), T(0), T(FFTH_S16_1), T(FFTH_SQRT_HALF), T(FFTH_C16_1)};
  const T s = c[(m + 12) & 15];  // sin(2 pi m/16) = cos(2 pi (m - 4)/16)
  return C2<T>{c[m & 15], DIR > 0 ? s : -s};
}

template <int R, int DIR, typename T> __device__ __forceinline__ void dft(C2<T>* a) {
  if constexpr (R == 2) {
    dft2<DIR>(a[0], a[1]);
  } else if constexpr (R == 3) {
    dft3<DIR>(a[0], a[1], a[2]);
  } else if constexpr (R == 4) {
    dft4<DIR>(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 5) {
    dft5<DIR>(a[0], a[1], a[2], a[3], a[4]);
  } else if constexpr (R == 8) {
    // 8 = 2 x 4: Y_s = DFT4(a[2m+s]); X[k2 + 4 k1] = sum_s w2^{k1 s} w8^{k2 s} Y_s[k2]
    dft4<DIR>(a[0], a[2], a[4], a[6]);
    dft4<DIR>(a[1], a[3], a[5], a[7]);
    C2<T> y1[4] = {a[1], cmul(a[3], w16<DIR, T>(2)), cmul(a[5], w16<DIR, T>(4)), cmul(a[7], w16<DIR, T>(6))};
    C2<T> y0[4] = {a[0], a[2], a[4], a[6]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = y0[k] + y1[k];
      a[k + 4] = y0[k] - y1[k];
    }
  } else if constexpr (R == 16) {
    // 16 = 4 x 4: Y_s = DFT4(a[4m+s]); twiddle w16^{k2 s}; X[k2 + 4 k1] = DFT4_s
    C2<T> y[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      C2<T> b0 = a[s], b1 = a[s + 4], b2 = a[s + 8], b3 = a[s + 12];
      dft4<DIR>(b0, b1, b2, b3);
      y[s][0] = b0;
      y[s][1] = s ? cmul(b1, w16<DIR, T>(s)) : b1;
      y[s][2] = s ? cmul(b2, w16<DIR, T>(2 * s)) : b2;
      y[s][3] = s ? cmul(b3, w16<DIR, T>(3 * s)) : b3;
    }
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      C2<T> b0 = y[0][k2], b1 = y[1][k2], b2 = y[2][k2], b3 = y[3][k2];
      dft4<DIR>(b0, b1, b2, b3);
      a[k2] = b0;
      a[k2 + 4] = b1;
      a[k2 + 8] = b2;
      a[k2 + 12] = b3;
    }
  }
}

// ---------------------------------------------------------------------------
// Twiddle table w[m] = exp(-2 pi i m / N), m in [0, N), built in LDS from
// sincospi in FP64 (then rounded to T).
// ---------------------------------------------------------------------------
template <typename T, int N, int NT> __device__ __forceinline__ void build_twiddles(C2<T>* tw) {
  for (int m = threadIdx.x; m < N; m += NT) {
    double s, c;
    sincospi(-2.0 * (double)m / (double)N, &s, &c);
    tw[m] = C2<T>{(T)c, (T)s};
  }
}

// ---------------------------------------------------------------------------
// Batched in-place Stockham FFT in LDS.
//   NFFT sequences of length N; element e of sequence f is at
//   buf[f*FS + PAD(e*ES)] where PAD inserts one slot every 16 when PADDED.
//   FFAST: consecutive threads take consecutive sequences (strided layouts);
//   otherwise consecutive butterflies of one sequence (contiguous layouts).
// Every stage: all reads to registers, barrier, all writes, barrier.
// ---------------------------------------------------------------------------
template <bool PADDED> __device__ __forceinline__ int padx(int e) { return PADDED ? e + (e >> 4) : e; }

// Spectrum values in global memory: full-precision complex, or a pair of
// binary16 values (round to nearest on store, exact widening on load).
struct H2 {
  _Float16 x, y;
};
template <typename T> __device__ __forceinline__ C2<T> sload(const C2<T>* p) { return *p; }
template <typename T> __device__ __forceinline__ C2<T> sload(const H2* p) {
  const H2 h = *p;
  return C2<T>{(T)h.x, (T)h.y};
}
template <typename T> __device__ __forceinline__ void sstore(C2<T>* p, const C2<T>& v) { *p = v; }
template <typename T> __device__ __forceinline__ void sstore(H2* p, const C2<T>& v) {
  *p = H2{(_Float16)v.x, (_Float16)v.y};
}

// Two adjacent complex values moved with one 16-byte access (FP32 layouts in
// which consecutive sequences are adjacent in memory).
template <typename T> struct alignas(16) Pair { C2<T> a, b; };

template <typename T, int V> __device__ __forceinline__ void load_v(const C2<T>* p, C2<T> (&o)[V]) {
  if constexpr (V == 2) {
    const Pair<T> q = *reinterpret_cast<const Pair<T>*>(p);
    o[0] = q.a;
    o[1] = q.b;
  } else {
    o[0] = p[0];
  }
}
template <typename T, int V> __device__ __forceinline__ void store_v(C2<T>* p, const C2<T> (&o)[V]) {
  if constexpr (V == 2) {
    *reinterpret_cast<Pair<T>*>(p) = Pair<T>{o[0], o[1]};
  } else {
    p[0] = o[0];
  }
}

// G adjacent binary16 complex values moved with one access of 4 G bytes
// (p aligned to that size).
template <int G> struct alignas(4 * G) H2G { H2 h[G]; };
template <typename T, int G> __device__ __forceinline__ void hload_g(const H2* p, C2<T> (&o)[G]) {
  const H2G<G> q = *reinterpret_cast<const H2G<G>*>(p);
#pragma unroll
  for (int i = 0; i < G; ++i) o[i] = C2<T>{(T)q.h[i].x, (T)q.h[i].y};
}
template <typename T, int G> __device__ __forceinline__ void hstore_g(H2* p, const C2<T> (&o)[G]) {
  H2G<G> q;
#pragma unroll
  for (int i = 0; i < G; ++i) q.h[i] = H2{(_Float16)o[i].x, (_Float16)o[i].y};
  *reinterpret_cast<H2G<G>*>(p) = q;
}


// One Stockham stage.  Work items are (group of V adjacent sequences, butterfly).
// V = 2 requires FFAST layouts with sequence stride FS = 1 (adjacent sequences).
template <typename T, int N, int S, int NFFT, int NT, int ES, int FS, bool FFAST, bool PADDED, int DIR, int V,
          int PLAN = 0>
__device__ __forceinline__ void fft_stage(C2<T>* buf, const C2<T>* tw) {
  static_assert(V == 1 || (FFAST && FS == 1 && NFFT % V == 0 && ES % V == 0), "vector width needs adjacent sequences");
  constexpr int R = fac_radix(N, S, PLAN);
  constexpr int NS = fac_prefix(N, S, PLAN);
  constexpr int NB = N / R;
  constexpr int NG = NFFT / V;
  constexpr int ITEMS = NG * NB;
  constexpr int K = (ITEMS + NT - 1) / NT;
  C2<T> v[K][V][R];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int it = threadIdx.x + k * NT;
    if ((ITEMS % NT == 0) || it < ITEMS) {
      const int g = FFAST ? it % NG : it / NB;
      const int j = FFAST ? it / NG : it % NB;
      const C2<T>* src = buf + g * V * FS;
      const int kk = j % NS;
      // radix 4, 8, 16: the twiddles w^r, r = 1..R-1, from w, w^2, w^4, ...
      // (log2 R table reads) by at most log2 R - 1 products each
      constexpr int LB = R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 0;
      constexpr bool POW = LB > 0;
      C2<T> wp[LB > 0 ? LB : 1];
      if constexpr (POW && NS > 1) {
#pragma unroll
        for (int b = 0; b < LB; ++b) {
          wp[b] = tw[(1 << b) * kk * (N / (NS * R))];
          if (DIR > 0) wp[b].y = -wp[b].y;
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C2<T> a[V];
        load_v<T, V>(src + padx<PADDED>((j + r * NB) * ES), a);
        if (NS > 1 && r > 0) {
          C2<T> w;
          if constexpr (POW) {
            bool have = false;
#pragma unroll
            for (int b = 0; b < LB; ++b) {
              if (r & (1 << b)) {
                w = have ? cmul(w, wp[b]) : wp[b];
                have = true;
              }
            }
          } else {
            w = tw[r * kk * (N / (NS * R))];
            if (DIR > 0) w.y = -w.y;
          }
#pragma unroll
          for (int q = 0; q < V; ++q) a[q] = cmul(a[q], w);
        }
#pragma unroll
        for (int q = 0; q < V; ++q) v[k][q][r] = a[q];
      }
#pragma unroll
      for (int q = 0; q < V; ++q) dft<R, DIR>(v[k][q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int it = threadIdx.x + k * NT;
    if ((ITEMS % NT == 0) || it < ITEMS) {
      const int g = FFAST ? it % NG : it / NB;
      const int j = FFAST ? it / NG : it % NB;
      C2<T>* dst = buf + g * V * FS;
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C2<T> a[V];
#pragma unroll
        for (int q = 0; q < V; ++q) a[q] = v[k][q][r];
        store_v<T, V>(dst + padx<PADDED>((base + r * NS) * ES), a);
      }
    }
  }
  __syncthreads();
}

template <typename T, int N, int S, int NFFT, int NT, int ES, int FS, bool FFAST, bool PADDED, int DIR, int V,
          int PLAN>
__device__ __forceinline__ void fft_stages(C2<T>* buf, const C2<T>* tw) {
  if constexpr (S < fac_count(N, PLAN)) {
    fft_stage<T, N, S, NFFT, NT, ES, FS, FFAST, PADDED, DIR, V, PLAN>(buf, tw);
    fft_stages<T, N, S + 1, NFFT, NT, ES, FS, FFAST, PADDED, DIR, V, PLAN>(buf, tw);
  }
}

// Caller must __syncthreads() before (data written) - the stages end with a barrier.
template <typename T, int N, int NFFT, int NT, int ES, int FS, bool FFAST, bool PADDED, int DIR, int V = 1,
          int PLAN = 0>
__device__ __forceinline__ void lds_fft(C2<T>* buf, const C2<T>* tw) {
  static_assert(fac_count(N, PLAN) > 0, "unsupported FFT length");
  fft_stages<T, N, 0, NFFT, NT, ES, FS, FFAST, PADDED, DIR, V, PLAN>(buf, tw);
}

// ---------------------------------------------------------------------------
// Reductions: NR double sums per block, fixed order (deterministic).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// out[r * stride] = block sum of v[r] (stride 1: NR consecutive doubles; stride =
// number of blocks: slot-major partial arrays).
template <int NR, int NT>
__device__ __forceinline__ void block_sums(double (&v)[NR], double* out, long stride = 1) {
  __shared__ double red[NT / 64][NR];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();  // red may still be read by a previous call
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    double s = wave_sum(v[r]);
    if (lane == 0) red[w][r] = s;
  }
  __syncthreads();
  if (threadIdx.x < NR) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i][threadIdx.x];
    out[threadIdx.x * stride] = s;
  }
}

}  // namespace ffth
