// libffth host driver: plans, workspace layout, the Basic Scheme / CG /
// mixed-precision solve loops, the order-1 right-hand side, and the C-ABI
// declared in include/ffth.h.
//
// Every step of the iteration runs in the HIP kernels of this library; the
// host only queues launches, uploads small descriptor/state structs and reads
// the per-load convergence flags every `check_every` iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <deque>
#include <tuple>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "admission.h"
#include "arena.h"
#include "desc_check.h"
#include "ffth.h"
#include "ffth_launch.h"
#include "ffth_types.h"

using namespace ffth;

namespace {

thread_local std::string g_last_error;

constexpr int NRED_ = NRED;
constexpr int MS_BLOCKS_MAX = 1024;   // blocks of the pointwise reduction kernels
constexpr int NT = 256;              // threads per block of the pointwise kernels
constexpr size_t ALIGN = 256;

size_t al(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}
#define HIPCHK(call)                                  \
  do {                                                \
    if (!hip_ok((call), #call)) return FFTH_ERR_DEVICE; \
  } while (0)

// Workspace regions (byte offsets).  Computed identically for sizing and
// for carving a caller's buffer.
struct Layout {
  size_t mat64, mat32, desc, cdesc, state, part, spec, f32, f64, P, X1, X2, g, misc, total;
  size_t spec_stride, f32_stride, f64_stride, part_stride;
  int nf32, nf64;
  int ndesc, nstate, nblk;
};

int x_blocks(int n0, int n1, int n2, bool dbl, bool inverse, int v) {
  const long rows = (long)n0 * n1;
  const int r = inverse ? (dbl ? Launch<double>::xi_rows(n2, v) : Launch<float>::xi_rows(n2, v))
                        : (dbl ? Launch<double>::x_rows(n2, v) : Launch<float>::x_rows(n2, v));
  return r > 0 ? (int)((rows + r - 1) / r) : 0;
}

int ms_blocks(long nvox) { return (int)std::min<long>(MS_BLOCKS_MAX, (nvox + NT - 1) / NT); }

Layout make_layout(const int n[3], int nph, int nloads, int order, const ffth_opts& o) {
  Layout L{};
  const long nvox = (long)n[0] * n[1] * n[2];
  const int prec = o.precision, scheme = o.scheme;
  L.ndesc = 7 * nloads + 8;
  L.nstate = 3 * nloads + 1;
  L.nblk = std::max((int)((long)n[0] * n[1]), ms_blocks(nvox));   // x-pass blocks of any variant (>= 1 row)
  // per-load FP32 / FP64 field counts
  // three-term CG (the mixed inner solve and FFTH_CG3): x, r in two slots each
  if (prec == FFTH_FP32) L.nf32 = scheme == FFTH_CG ? 3 : scheme == FFTH_BICGSTAB ? 7 : scheme == FFTH_CG3 ? 4 : 1;
  if (prec == FFTH_MIXED) L.nf32 = scheme == FFTH_CG ? 4 : 2;
  if (prec == FFTH_FP64) L.nf64 = scheme == FFTH_CG ? 2 : scheme == FFTH_BICGSTAB ? 6 : scheme == FFTH_CG3 ? 4 : 0;
  if (prec == FFTH_MIXED) L.nf64 = 1;   // FP64 residual before its compatible projection
  L.spec_stride = al((size_t)nvox * 6 * sizeof(double));     // 6 x (nvox/2) complex FP64
  L.f32_stride = al((size_t)nvox * 6 * sizeof(float));
  L.f64_stride = al((size_t)nvox * 6 * sizeof(double));
  L.part_stride = al((size_t)L.nblk * NRED_ * sizeof(double));
  size_t off = 0;
  L.mat64 = off; off += al((size_t)nph * 72 * sizeof(double));
  L.mat32 = off; off += al((size_t)nph * 72 * sizeof(float));
  L.desc = off; off += al((size_t)L.ndesc * sizeof(Desc));
  L.cdesc = off; off += al((size_t)4 * nloads * sizeof(Desc));   // compacted active-load copies
  L.state = off; off += al((size_t)L.nstate * sizeof(SolverState));
  L.misc = off; off += ALIGN;
  L.part = off; off += (size_t)(2 * nloads + 2) * L.part_stride;
  L.spec = off; off += (size_t)nloads * L.spec_stride;
  L.f32 = off; off += (size_t)nloads * L.nf32 * L.f32_stride;
  L.f64 = off; off += (size_t)nloads * L.nf64 * L.f64_stride;
  L.P = off;
  if (order >= 1) off += (size_t)nloads * L.f64_stride;
  L.X1 = off;                                   // order-0 corrector displacements [6][3][N]
  if (order >= 1) off += al((size_t)nvox * 18 * sizeof(double));
  L.X2 = off;                                   // order-1 unit-gradient displacements [18][3][N]
  if (order == 2) off += al((size_t)nvox * 54 * sizeof(double));
  L.g = off;
  if (order >= 1) off += (size_t)nloads * al((size_t)nvox * 3 * sizeof(double));
  L.total = off;
  return L;
}

bool opts_valid(const ffth_opts& o) {
  if (o.scheme != FFTH_BASIC && o.scheme != FFTH_CG && o.scheme != FFTH_BICGSTAB && o.scheme != FFTH_CG3) return false;
  // FP64 or FP32 only
  if ((o.scheme == FFTH_BICGSTAB || o.scheme == FFTH_CG3) && o.precision == FFTH_MIXED) return false;
  if (o.precision < FFTH_FP64 || o.precision > FFTH_MIXED) return false;
  if (!(o.tol > 0.0) || o.max_iter < 1 || o.check_every < 1) return false;
  if (o.precision == FFTH_MIXED && (!(o.inner_tol > 0.0) || o.inner_tol >= 1.0 || o.max_outer < 1)) return false;
  if (o.spectrum16 < 0 || o.spectrum16 > 2) return false;
  return true;
}

void voigt21_to_m(const double* v21, double m[36]) {
  double c[6][6];
  int k = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b) c[a][b] = c[b][a] = v21[k++];
  // sigma_a = sum_b C_ab * eps_eng_b, eps_eng_b = eps_b (b < 3) or 2 eps_b (shear)
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) m[a * 6 + b] = c[a][b] * (b < 3 ? 1.0 : 2.0);
}

void iso_to_m(double lam, double mu, double m[36]) {
  for (int i = 0; i < 36; ++i) m[i] = 0.0;
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) m[a * 6 + b] = lam;
    m[a * 6 + a] += 2.0 * mu;
  }
  for (int a = 3; a < 6; ++a) m[a * 6 + a] = 2.0 * mu;
}

// Eigenvalues of a symmetric 6 x 6 matrix (cyclic Jacobi rotations).
void sym6_eigenvalues(double a[6][6], double ev[6]) {
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) (i == j ? tot : off) += a[i][j] * a[i][j];
    if (off <= 1e-30 * (tot + off)) break;
    for (int p = 0; p < 5; ++p) {
      for (int q = p + 1; q < 6; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 6; ++k) {   // A <- A J
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 6; ++k) {   // A <- J^T A
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
      }
    }
  }
  for (int i = 0; i < 6; ++i) ev[i] = a[i][i];
}

// Stiffness contrast of the phases: the largest eigen-modulus (eigenvalue of
// the stiffness in Mandel form) over the smallest, across all phases; infinite
// when a phase is not positive definite.  Isotropic phases have 3 lambda + 2 mu
// (once) and 2 mu (five times).
double stiffness_contrast(int nph, bool iso, const double* lame, const double* v21) {
  double lo = INFINITY, hi = 0.0;
  for (int ph = 0; ph < nph; ++ph) {
    double ev[6];
    if (iso) {
      const double lam = lame[2 * ph], mu = lame[2 * ph + 1];
      ev[0] = 3.0 * lam + 2.0 * mu;
      for (int i = 1; i < 6; ++i) ev[i] = 2.0 * mu;
    } else {
      double a[6][6];
      int k = 0;
      for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) {
          const double w = (r < 3 ? 1.0 : std::sqrt(2.0)) * (c < 3 ? 1.0 : std::sqrt(2.0));
          a[r][c] = a[c][r] = v21[21 * ph + k++] * w;
        }
      sym6_eigenvalues(a, ev);
    }
    for (int i = 0; i < 6; ++i) {
      if (!(ev[i] == ev[i])) return NAN;   // a coefficient that is not a number
      lo = std::min(lo, ev[i]);
      hi = std::max(hi, ev[i]);
    }
  }
  return lo > 0.0 ? hi / lo : INFINITY;
}

}  // namespace

void ffth::set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

// Pinned host buffers that are handed out again instead of freed: freeing
// pinned memory synchronizes the whole device, which in a server would stall
// every stream each time a request finishes.  Sizes are rounded up to powers
// of two (at least 4 KiB); a plan created with a pool returns its buffers to
// it when destroyed, and the pool frees them all when released.
struct HostPool {
  std::map<size_t, std::vector<void*>> free_;
  std::vector<void*> all;
  static size_t rounded(size_t b) {
    size_t r = 4096;
    while (r < b) r <<= 1;
    return r;
  }
  void* get(size_t bytes) {
    std::vector<void*>& v = free_[rounded(bytes)];
    if (!v.empty()) {
      void* q = v.back();
      v.pop_back();
      return q;
    }
    void* q = nullptr;
    if (hipHostMalloc(&q, rounded(bytes), hipHostMallocDefault) != hipSuccess) return nullptr;
    all.push_back(q);
    return q;
  }
  void put(void* q, size_t bytes) {
    if (q) free_[rounded(bytes)].push_back(q);
  }
  void release() {
    for (void* q : all) (void)hipHostFree(q);
    all.clear();
    free_.clear();
  }
};

struct ffth_plan {
  int n[3];
  long nvox;
  int h;
  long rows;
  int nph;
  bool iso;
  double lam0, mu0;
  bool h16 = false;    // the mixed scheme's FP32 inner solve keeps its spectrum in binary16
  double kappa = 1.0;  // max row sum of |C - C0| / mu0 over the phases (range of the polarization)
  double contrast = 1.0;  // largest over smallest eigen-modulus of the phases
  const uint16_t* phase;
  hipStream_t stream;
  int nloads;
  int order;
  ffth_opts opts;
  char* ws;
  Layout L;
  double* mat64;
  float* mat32;
  Desc* d_desc;
  SolverState* d_state;
  SolverState* h_state;   // pinned host mirror (read-back)
  Desc* d_cdesc;          // 4 regions of nloads compacted descriptors
  Desc* h_cdesc;          // pinned staging for them
  HostPool* hpool = nullptr;   // where h_state and h_cdesc come from (null: hipHostMalloc / hipHostFree)
  int nx64, nx32;         // forward x-pass blocks per precision
  int ni64, ni32;         // inverse x-pass blocks per precision
  int var[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};   // tile variant per pass (xf, y, z, xi) and FP32/FP64
  int bw[2] = {0, 0};     // loads per launch of the iteration passes, FP32/FP64 (0: all at once)
  std::vector<Desc> h_desc;
  // kernel timing (diagnostics): events bracket every launch when enabled
  bool prof = false;
  struct Rec { int cat, units; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double prof_ms[16] = {0};
  long prof_n[16] = {0};
  long prof_units[16] = {0};   // batch entries (loads) processed, summed over launches
};

namespace {

void set_blocks(ffth_plan* P) {
  P->nx32 = x_blocks(P->n[0], P->n[1], P->n[2], false, false, P->var[0][0]);
  P->nx64 = x_blocks(P->n[0], P->n[1], P->n[2], true, false, P->var[0][1]);
  P->ni32 = x_blocks(P->n[0], P->n[1], P->n[2], false, true, P->var[3][0]);
  P->ni64 = x_blocks(P->n[0], P->n[1], P->n[2], true, true, P->var[3][1]);
}

double* part_ptr(ffth_plan* P, int slot) { return (double*)(P->ws + P->L.part + (size_t)slot * P->L.part_stride); }
void* spec_ptr(ffth_plan* P, int l) { return P->ws + P->L.spec + (size_t)l * P->L.spec_stride; }
float* f32_ptr(ffth_plan* P, int l, int k) {
  return (float*)(P->ws + P->L.f32 + ((size_t)l * P->L.nf32 + k) * P->L.f32_stride);
}
double* f64_ptr(ffth_plan* P, int l, int k) {
  return (double*)(P->ws + P->L.f64 + ((size_t)l * P->L.nf64 + k) * P->L.f64_stride);
}
double* Pfield(ffth_plan* P, int l) { return (double*)(P->ws + P->L.P + (size_t)l * P->L.f64_stride); }
double* X1field(ffth_plan* P) { return (double*)(P->ws + P->L.X1); }
double* X2field(ffth_plan* P) { return (double*)(P->ws + P->L.X2); }
double* gfield(ffth_plan* P, int l) {
  return (double*)(P->ws + P->L.g + (size_t)l * al((size_t)P->nvox * 3 * sizeof(double)));
}

// State slots: [0, nl) main/outer, [nl, 2nl) inner, [2nl, 3nl) post/utility, 3nl spare utility.
SolverState* st_main(ffth_plan* P, int l) { return P->d_state + l; }
SolverState* st_inner(ffth_plan* P, int l) { return P->d_state + P->nloads + l; }
SolverState* st_post(ffth_plan* P, int l) { return P->d_state + 2 * P->nloads + l; }

// Descriptor slots (roles x nloads).
enum Role { R_MAIN = 0, R_MAIN_DELTA = 1, R_INNER = 2, R_POST = 3, R_THETA = 4, R_UTIL = 5, R_PROJ = 6 };
int desc_slot(ffth_plan* P, Role r, int l) { return (int)r * P->nloads + l; }
const Desc* dptr(ffth_plan* P, Role r) { return P->d_desc + desc_slot(P, r, 0); }
// the 6 order-1 displacement descriptors live after the role blocks
int util6_slot(ffth_plan* P, int J) { return 7 * P->nloads + J; }

// ---- kernel timing ---------------------------------------------------------
enum Cat {
  C_XF32 = 0, C_Y32, C_Z32, C_XI32, C_XF64, C_Y64, C_Z64, C_XI64, C_FIN, C_POINT, C_XCG3, C_CG3S, C_XCG3_64,
  C_CG3S_64, NCAT
};
const char* const CAT_NAMES[NCAT] = {"xfwd_f32", "ypass_f32", "zpass_f32", "xinv_f32", "xfwd_f64",
                                     "ypass_f64", "zpass_f64", "xinv_f64", "finalize", "pointwise",
                                     "xcg3_f32", "cg3start_f32", "xcg3_f64", "cg3start_f64"};

hipEvent_t take_event(ffth_plan* P) {
  if (P->pool.empty()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = P->pool.back();
  P->pool.pop_back();
  return e;
}

// Bracket one launch: call before (returns the record index or -1) and after.
int prof_begin(ffth_plan* P, int cat, int units) {
  if (!P->prof) return -1;
  ffth_plan::Rec r{cat, units, take_event(P), take_event(P)};
  if (!r.a || !r.b) return -1;
  (void)hipEventRecord(r.a, P->stream);
  P->recs.push_back(r);
  return (int)P->recs.size() - 1;
}
void prof_end(ffth_plan* P, int idx) {
  if (idx >= 0) (void)hipEventRecord(P->recs[idx].b, P->stream);
}
// Called after a stream synchronisation: fold finished records into the totals.
void prof_flush(ffth_plan* P) {
  for (auto& r : P->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      P->prof_ms[r.cat] += ms;
      P->prof_n[r.cat] += 1;
      P->prof_units[r.cat] += r.units;
    }
    P->pool.push_back(r.a);
    P->pool.push_back(r.b);
  }
  P->recs.clear();
}

struct ProfScope {
  ffth_plan* P;
  int idx;
  ProfScope(ffth_plan* p, int cat, int units) : P(p), idx(prof_begin(p, cat, units)) {}
  ~ProfScope() { prof_end(P, idx); }
};

Desc base_desc(ffth_plan* P, int l) {
  Desc d;
  std::memset(&d, 0, sizeof(d));
  d.phase = P->phase;
  d.mat64 = P->mat64;
  d.mat32 = P->mat32;
  d.spec = spec_ptr(P, l);
  d.part_f = part_ptr(P, 2 * l);
  d.part_i = part_ptr(P, 2 * l + 1);
  d.lam0 = P->lam0;
  d.mu0 = P->mu0;
  d.nc = 6;
  d.inv_nvox = 1.0 / (double)P->nvox;
  d.tau_scale = 1.0;
  d.op_scale = 1.0 / (double)P->nvox;
  for (int a = 0; a < 3; ++a) d.n[a] = P->n[a];
  return d;
}

SolverState make_state(double tol, int max_iter, double guard_eps, int active) {
  SolverState s;
  std::memset(&s, 0, sizeof(s));
  s.tol = tol;
  s.tol0 = tol;
  s.max_iter = max_iter;
  s.guard_eps = guard_eps;
  s.gscale = -1.0;
  s.active = active;
  s.first = 1;
  s.res = 1.0;
  s.dscale = 1.0;
  return s;
}

ffth_status upload_descs(ffth_plan* P) {
  HIPCHK(hipMemcpyAsync(P->d_desc, P->h_desc.data(), P->h_desc.size() * sizeof(Desc), hipMemcpyHostToDevice,
                        P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  return FFTH_OK;
}

ffth_status upload_states(ffth_plan* P, const std::vector<SolverState>& s, int first_slot) {
  HIPCHK(hipMemcpyAsync(P->d_state + first_slot, s.data(), s.size() * sizeof(SolverState), hipMemcpyHostToDevice,
                        P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  std::memcpy(P->h_state + first_slot, s.data(), s.size() * sizeof(SolverState));  // keep the mirror current
  return FFTH_OK;
}

ffth_status read_states(ffth_plan* P) {
  HIPCHK(hipMemcpyAsync(P->h_state, P->d_state, P->L.nstate * sizeof(SolverState), hipMemcpyDeviceToHost,
                        P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  prof_flush(P);
  return FFTH_OK;
}

// ---- pass launchers -------------------------------------------------------

enum Pass { PS_XF = 0, PS_Y = 1, PS_Z = 2, PS_XI = 3 };
template <typename T> int pv(ffth_plan* P, Pass ps) { return P->var[ps][sizeof(T) == 8 ? 1 : 0]; }

template <typename T> int xblocks(ffth_plan* P) { return sizeof(T) == 8 ? P->nx64 : P->nx32; }
template <typename T> int iblocks(ffth_plan* P) { return sizeof(T) == 8 ? P->ni64 : P->ni32; }
// Loads per launch of the iteration passes for an iteration over nb loads:
// all of them, unless the plan's width for this precision is smaller.
template <typename T> int chunk_of(ffth_plan* P, int nb) {
  const int w = P->bw[sizeof(T) == 8 ? 1 : 0];
  return w > 0 && w < nb ? w : nb;
}

template <typename T> ffth_status xfwd(ffth_plan* P, const Desc* d, int nb, int mode, bool h16 = false) {
  ProfScope ps(P, mode == XF_R3 ? (sizeof(T) == 8 ? C_CG3S_64 : C_CG3S) : sizeof(T) == 8 ? C_XF64 : C_XF32, nb);
  HIPCHK(Launch<T>::xfwd(P->n[2], P->iso, pv<T>(P, PS_XF), h16, dim3(xblocks<T>(P), nb), P->stream, d, mode, P->rows,
                         P->nvox));
  return FFTH_OK;
}

// Half spectrum layout [h/kc][n0][n1][kc][6]: the y-pass sees n0*h/kc planes of
// [n1][kc*6]; the z-pass sees h/kc chunks of [n0][n1*kc][6].
int kchunk_host(int h) {
  int c = h < 16 ? h : 16;
  while (h % c) --c;
  return c;
}

template <typename T> ffth_status yzy(ffth_plan* P, const Desc* d, int nb, int op, bool h16 = false) {
  const int kc = kchunk_host(P->h);
  const int ncols = kc * 6;
  const int nplanes = P->n[0] * (P->h / kc);
  const int vy = pv<T>(P, PS_Y), vz = pv<T>(P, PS_Z);
  const int cw = Launch<T>::y_cols(P->n[1], vy);
  const int ntiles = (ncols + cw - 1) / cw;
  const int cy = sizeof(T) == 8 ? C_Y64 : C_Y32, cz = sizeof(T) == 8 ? C_Z64 : C_Z32;
  {
    ProfScope ps(P, cy, nb);
    HIPCHK(Launch<T>::ypass(P->n[1], vy, h16, dim3(nplanes * ntiles, nb), P->stream, d, -1, ncols, ntiles));
  }
  const long M = (long)P->n[1] * kc;
  const int tk = Launch<T>::z_cols(P->n[0], vz);
  const double scale = 1.0 / (double)P->nvox;
  {
    ProfScope ps(P, cz, nb);
    const int nzb = (int)((M + tk - 1) / tk) * (P->h / kc);
    HIPCHK(Launch<T>::zpass(P->n[0], vz, h16, dim3(nzb, nb), P->stream, d, op, P->n[1], P->h, scale));
  }
  {
    ProfScope ps(P, cy, nb);
    // the inverse y-transform reads the FP32 copy of a binary16 inner solve
    HIPCHK(Launch<T>::ypass(P->n[1], vy, false, dim3(nplanes * ntiles, nb), P->stream, d, +1, ncols, ntiles));
  }
  return FFTH_OK;
}

template <typename T> ffth_status xinv(ffth_plan* P, const Desc* d, int nb, int mode) {
  ProfScope ps(P, sizeof(T) == 8 ? C_XI64 : C_XI32, nb);
  HIPCHK(Launch<T>::xinv(P->n[2], P->iso, pv<T>(P, PS_XI), dim3(iblocks<T>(P), nb), P->stream, d, mode, P->rows,
                         P->nvox));
  return FFTH_OK;
}

ffth_status fin(ffth_plan* P, const Desc* d, int nb, int op, int nblk_f, int nblk_i) {
  ProfScope ps(P, C_FIN, nb);
  HIPCHK(launch_finalize(nb, P->stream, d, op, nblk_f, nblk_i));
  return FFTH_OK;
}

// Start of a three-term CG solve: tau(r_0), its x-transform and the scalars.
// h16: the binary16-spectrum kernels (FP32 inner solves of a binary16 plan).
template <typename T> ffth_status cg3_start(ffth_plan* P, const Desc* d, int nb, bool h16) {
  ffth_status s;
  if (nb <= 0) return FFTH_OK;
  if ((s = xfwd<T>(P, d, nb, XF_R3, h16)) != FFTH_OK) return s;
  return fin(P, d, nb, FIN_CG3_INIT, xblocks<T>(P), 0);
}

// One three-term CG iteration: y, z (Green operator), y, fused x-pass (per
// group of chunk_of loads), then the scalars of every load.
template <typename T> ffth_status cg3_iter(ffth_plan* P, const Desc* d, int nb, bool h16) {
  ffth_status s;
  if (nb <= 0) return FFTH_OK;
  const int c = chunk_of<T>(P, nb);
  for (int i = 0; i < nb; i += c) {
    const int k = std::min(c, nb - i);
    if ((s = yzy<T>(P, d + i, k, OP_GAMMA, h16)) != FFTH_OK) return s;
    ProfScope ps(P, sizeof(T) == 8 ? C_XCG3_64 : C_XCG3, k);
    HIPCHK(Launch<T>::xcg3(P->n[2], P->iso, pv<T>(P, PS_XI), h16, dim3(iblocks<T>(P), k), P->stream, d + i, P->rows,
                           P->nvox));
  }
  return fin(P, d, nb, FIN_CG3, 0, iblocks<T>(P));
}

// ---- autotuner ------------------------------------------------------------
//
// Each pass has NVAR compiled tile shapes.  At plan creation every variant of
// every pass the plan will run is timed on the plan's own workspace (HIP
// events on its stream, in the modes the solver uses) and the fastest kept.
// Choices are cached per (grid, material kind, precision, scheme) for the
// process.  Grids below 64^3 keep the defaults (launch-bound).
std::mutex g_tune_mu;
std::map<std::array<int, 7>, std::array<int, 10>> g_tune_cache;   // tiles [8], loads per launch [2]

template <class F> double time_launches(hipStream_t st, hipEvent_t e0, hipEvent_t e1, F&& launch) {
  launch();  // warm-up
  (void)hipEventRecord(e0, st);
  launch();
  (void)hipEventRecord(e1, st);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  const int reps = std::max(3, std::min(50, (int)std::ceil(6.0 / std::max(ms, 1e-3f))));
  (void)hipEventRecord(e0, st);
  for (int i = 0; i < reps; ++i) launch();
  (void)hipEventRecord(e1, st);
  (void)hipEventSynchronize(e1);
  (void)hipEventElapsedTime(&ms, e0, e1);
  return ms / reps;
}

template <typename T>
void tune_prec(ffth_plan* P, const Desc* d, int nt, int xf_mode, int xi_mode, bool fused, bool h16) {
  const int pi = sizeof(T) == 8 ? 1 : 0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return;
  }
  const int kc = kchunk_host(P->h);
  const int ncols = kc * 6, nplanes = P->n[0] * (P->h / kc);
  const long M = (long)P->n[1] * kc;
  for (int pass = 0; pass < 4; ++pass) {
    double best = 1e30;
    int bv = 0;
    for (int v = 0; v < NVAR; ++v) {
      P->var[pass][pi] = v;
      set_blocks(P);
      double t;
      if (pass == PS_XF) {
        t = time_launches(P->stream, e0, e1, [&] {
          (void)Launch<T>::xfwd(P->n[2], P->iso, v, h16, dim3(xblocks<T>(P), nt), P->stream, d, xf_mode, P->rows,
                                P->nvox);
        });
      } else if (pass == PS_Y) {
        const int cw = Launch<T>::y_cols(P->n[1], v), ntl = (ncols + cw - 1) / cw;
        // binary16 forward spectrum: the variant serves the binary16 forward and
        // the FP32 inverse transform, so both are timed together
        t = time_launches(P->stream, e0, e1, [&] {
          (void)Launch<T>::ypass(P->n[1], v, h16, dim3(nplanes * ntl, nt), P->stream, d, -1, ncols, ntl);
          if (h16) (void)Launch<T>::ypass(P->n[1], v, false, dim3(nplanes * ntl, nt), P->stream, d, +1, ncols, ntl);
        });
      } else if (pass == PS_Z) {
        const int tk = Launch<T>::z_cols(P->n[0], v);
        const int nzb = (int)((M + tk - 1) / tk) * (P->h / kc);
        t = time_launches(P->stream, e0, e1, [&] {
          (void)Launch<T>::zpass(P->n[0], v, h16, dim3(nzb, nt), P->stream, d, OP_GAMMA, P->n[1], P->h,
                                 1.0 / (double)P->nvox);
        });
      } else if (fused) {
        t = time_launches(P->stream, e0, e1, [&] {
          (void)Launch<T>::xcg3(P->n[2], P->iso, v, h16, dim3(iblocks<T>(P), nt), P->stream, d, P->rows, P->nvox);
        });
      } else {
        t = time_launches(P->stream, e0, e1, [&] {
          (void)Launch<T>::xinv(P->n[2], P->iso, v, dim3(iblocks<T>(P), nt), P->stream, d, xi_mode, P->rows, P->nvox);
        });
      }
      if (t < best * (v == 0 ? 1.0 : 0.98)) {   // a variant must beat the default by 2%
        best = t;
        bv = v;
      }
    }
    P->var[pass][pi] = bv;
  }
  set_blocks(P);
  // loads per launch, with the chosen tiles: one whole iteration (x-forward
  // unless fused, y, z, y, x-inverse or the fused pass) over the nt loads,
  // all in one launch per pass, then w = 1, 2, 4, ... at a time, each group
  // through every pass before the next
  P->bw[pi] = 0;
  if (nt > 1) {
    const int cw = Launch<T>::y_cols(P->n[1], P->var[PS_Y][pi]), ntl = (ncols + cw - 1) / cw;
    const int tk = Launch<T>::z_cols(P->n[0], P->var[PS_Z][pi]);
    const int nzb = (int)((M + tk - 1) / tk) * (P->h / kc);
    auto iteration = [&](int w) {
      for (int i = 0; i < nt; i += w) {
        const int k = std::min(w, nt - i);
        if (!fused)
          (void)Launch<T>::xfwd(P->n[2], P->iso, P->var[PS_XF][pi], h16, dim3(xblocks<T>(P), k), P->stream, d + i,
                                xf_mode, P->rows, P->nvox);
        (void)Launch<T>::ypass(P->n[1], P->var[PS_Y][pi], h16, dim3(nplanes * ntl, k), P->stream, d + i, -1, ncols,
                               ntl);
        (void)Launch<T>::zpass(P->n[0], P->var[PS_Z][pi], h16, dim3(nzb, k), P->stream, d + i, OP_GAMMA, P->n[1],
                               P->h, 1.0 / (double)P->nvox);
        (void)Launch<T>::ypass(P->n[1], P->var[PS_Y][pi], false, dim3(nplanes * ntl, k), P->stream, d + i, +1, ncols,
                               ntl);
        if (fused)
          (void)Launch<T>::xcg3(P->n[2], P->iso, P->var[PS_XI][pi], h16, dim3(iblocks<T>(P), k), P->stream, d + i,
                                P->rows, P->nvox);
        else
          (void)Launch<T>::xinv(P->n[2], P->iso, P->var[PS_XI][pi], dim3(iblocks<T>(P), k), P->stream, d + i,
                                xi_mode, P->rows, P->nvox);
      }
    };
    double best = time_launches(P->stream, e0, e1, [&] { iteration(nt); });
    for (int w = 1; w < nt; w *= 2) {
      const double t = time_launches(P->stream, e0, e1, [&] { iteration(w); });
      if (t < best * 0.98) {   // a width must beat the one-launch iteration by 2%
        best = t;
        P->bw[pi] = w;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Inner-solve descriptor with a binary16 forward spectrum: tau / (kappa mu0 n2)
// before the x-transform, the forward y-transform divided by n1, and
// kappa mu0 / n0 in the spectral operator, whose FP32 output goes to spec2
// (placed after the binary16 spectrum inside the load's spectrum region).
void set_h16(const ffth_plan* P, Desc& d) {
  d.h16 = 1;
  d.spec2 = (char*)d.spec + al((size_t)P->nvox * 3 * sizeof(float));
  d.tau_scale = 1.0 / (P->kappa * P->mu0 * (double)P->n[2]);
  d.op_scale = P->kappa * P->mu0 / (double)P->n[0];
}

ffth_status autotune(ffth_plan* P) {
  const ffth_opts& o = P->opts;
  if (!o.autotune || P->nvox < 64L * 64 * 64) return FFTH_OK;
  const std::array<int, 7> key{P->n[0], P->n[1], P->n[2], P->iso ? 1 : 0, o.precision, o.scheme, P->h16 ? 1 : 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      for (int i = 0; i < 8; ++i) P->var[i / 2][i % 2] = it->second[i];
      P->bw[0] = it->second[8];
      P->bw[1] = it->second[9];
      set_blocks(P);
      return FFTH_OK;
    }
  }
  ffth_status s;
  // steady-state iterations (the fused CG pass in an odd iteration, which
  // reads and writes the x pair beside the residuals), and launches carrying
  // all of the plan's loads, each on its own workspace, as the solve's
  // launches do
  SolverState us = make_state(0, 1, 0, 1);
  us.first = 0;
  us.iters = 3;
  std::vector<SolverState> u(1, us);
  if ((s = upload_states(P, u, 3 * P->nloads)) != FFTH_OK) return s;
  const Desc* dd = dptr(P, R_UTIL);
  const int nt = P->nloads;
  const bool mixed = o.precision == FFTH_MIXED;
  if (o.precision != FFTH_FP64) {   // FP32 passes: the inner iteration (or the plain FP32 solve)
    int xf = XF_LS, xi = XI_BS;
    bool fused = false;
    if ((mixed && o.scheme == FFTH_CG) || o.scheme == FFTH_CG3) {   // three-term CG (inner) solve
      xf = XF_R3;
      fused = true;
    } else if (P->L.nf32 >= 3) {
      xf = XF_CG;
      xi = XI_CG;
    } else if (P->L.nf32 == 2) {
      xf = XF_MATVEC;
      xi = XI_BS_INNER;
    }
    for (int l = 0; l < nt; ++l) {
      Desc d = base_desc(P, l);
      d.st = P->d_state + 3 * P->nloads;
      d.x = f32_ptr(P, l, 0);
      if (fused) {
        d.r = f32_ptr(P, l, 1);
        d.x1 = f32_ptr(P, l, 2);
        d.r1 = f32_ptr(P, l, 3);
        if (P->h16) set_h16(P, d);
      } else if (P->L.nf32 >= 3) {
        d.r = f32_ptr(P, l, 1);
        d.p = f32_ptr(P, l, 2);
      } else if (P->L.nf32 == 2) {
        d.r = f32_ptr(P, l, 1);
      }
      P->h_desc[desc_slot(P, R_UTIL, l)] = d;
    }
    if ((s = upload_descs(P)) != FFTH_OK) return s;
    tune_prec<float>(P, dd, nt, xf, xi, fused, fused && P->h16);
  }
  if (mixed || (o.precision == FFTH_FP64 && P->L.nf64 >= 2)) {   // FP64 passes
    const bool cg3 = o.scheme == FFTH_CG3;
    const int xf = mixed ? XF_LS : cg3 ? XF_R3 : XF_CG, xi = mixed ? XI_RESID : XI_CG;
    for (int l = 0; l < nt; ++l) {
      Desc d = base_desc(P, l);
      d.st = P->d_state + 3 * P->nloads;
      d.x = f64_ptr(P, l, 0);
      if (mixed) {
        d.r = f32_ptr(P, l, 1);
        d.r_f32 = 1;
      } else if (cg3) {
        d.r = f64_ptr(P, l, 1);
        d.x1 = f64_ptr(P, l, 2);
        d.r1 = f64_ptr(P, l, 3);
      } else {
        d.r = f64_ptr(P, l, 0);
        d.p = f64_ptr(P, l, 1);
      }
      P->h_desc[desc_slot(P, R_UTIL, l)] = d;
    }
    if ((s = upload_descs(P)) != FFTH_OK) return s;
    tune_prec<double>(P, dd, nt, xf, xi, cg3, false);
  }
  HIPCHK(hipStreamSynchronize(P->stream));
  HIPCHK(hipGetLastError());
  std::array<int, 10> val;
  for (int i = 0; i < 8; ++i) val[i] = P->var[i / 2][i % 2];
  val[8] = P->bw[0];
  val[9] = P->bw[1];
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = val;
  return FFTH_OK;
}

// One full operator application: x-fwd(mode) [fin alpha] y z y x-inv(mode)
// per group of chunk_of loads, then fin(op) for all of them
template <typename T>
ffth_status apply(ffth_plan* P, const Desc* d, int nb, int xf, int spec_op, int xi, int fin_op) {
  ffth_status s;
  if (nb <= 0) return FFTH_OK;
  const int c = chunk_of<T>(P, nb);
  for (int i = 0; i < nb; i += c) {
    const int k = std::min(c, nb - i);
    if ((s = xfwd<T>(P, d + i, k, xf)) != FFTH_OK) return s;
    if (xf == XF_CG && (s = fin(P, d + i, k, FIN_CG_ALPHA, xblocks<T>(P), 0)) != FFTH_OK) return s;
    if ((s = yzy<T>(P, d + i, k, spec_op)) != FFTH_OK) return s;
    if ((s = xinv<T>(P, d + i, k, xi)) != FFTH_OK) return s;
  }
  if (fin_op >= 0 && (s = fin(P, d, nb, fin_op, xblocks<T>(P), iblocks<T>(P))) != FFTH_OK) return s;
  return FFTH_OK;
}

bool any_active(ffth_plan* P, int first, int count) {
  for (int i = 0; i < count; ++i)
    if (P->h_state[first + i].active) return true;
  return false;
}

// Launch set: the descriptors of role r for the loads whose state (slot
// state_base + l) was active at the last read-back, copied contiguously into
// compact region `region` so that grids span active loads only.  Loads that
// finish before the next read-back are still launched and exit at once.
struct DescSet {
  const Desc* d;
  int n;
};
DescSet active_set(ffth_plan* P, Role r, int state_base, int nl, int region) {
  Desc* stage = P->h_cdesc + (size_t)region * P->nloads;
  int k = 0;
  for (int l = 0; l < nl; ++l)
    if (P->h_state[state_base + l].active) stage[k++] = P->h_desc[desc_slot(P, r, l)];
  Desc* dst = P->d_cdesc + (size_t)region * P->nloads;
  if (k > 0 && !hip_ok(hipMemcpyAsync(dst, stage, k * sizeof(Desc), hipMemcpyHostToDevice, P->stream), "copy"))
    return DescSet{nullptr, -1};
  return DescSet{dst, k};
}

// ---- solve loops ----------------------------------------------------------

// One BiCGSTAB iteration (two operator applications): p and tau(p) [x-forward,
// applying the previous iteration's x and r updates], v = A p and <r^,v>,
// alpha; s = r - alpha v and tau(s), t = A s and the five sums, omega, beta.
template <typename T> ffth_status bicg_iter(ffth_plan* P, const Desc* d, int nb) {
  ffth_status s;
  if (nb <= 0) return FFTH_OK;
  const int c = chunk_of<T>(P, nb);
  for (int i = 0; i < nb; i += c) {   // per group of loads (load-major)
    const int k = std::min(c, nb - i);
    const Desc* g = d + i;
    if ((s = xfwd<T>(P, g, k, XF_BI1)) != FFTH_OK) return s;
    if ((s = yzy<T>(P, g, k, OP_GAMMA)) != FFTH_OK) return s;
    if ((s = xinv<T>(P, g, k, XI_BI1)) != FFTH_OK) return s;
    if ((s = fin(P, g, k, FIN_BI_ALPHA, 0, iblocks<T>(P))) != FFTH_OK) return s;
    if ((s = xfwd<T>(P, g, k, XF_BI2)) != FFTH_OK) return s;
    if ((s = yzy<T>(P, g, k, OP_GAMMA)) != FFTH_OK) return s;
    if ((s = xinv<T>(P, g, k, XI_BI2)) != FFTH_OK) return s;
  }
  return fin(P, d, nb, FIN_BI_OMEGA, 0, iblocks<T>(P));
}

// Iterate a plain (single precision level) scheme on descriptors d with
// states in slots [0, nl).  The iterate must hold zero on entry.
template <typename T> ffth_status run_cg3(ffth_plan* P, int nl);

template <typename T> ffth_status run_plain(ffth_plan* P, const Desc* d, int nl) {
  const ffth_opts& o = P->opts;
  ffth_status s;
  DescSet as;
  if (o.scheme == FFTH_CG3) return run_cg3<T>(P, nl);
  // pass 0: x = b = -Gamma0 * P_rhs, ||b||, zero right-hand-side guard
  if ((s = apply<T>(P, d, nl, XF_LS, OP_GAMMA, XI_BS, FIN_LS_FIRST)) != FFTH_OK) return s;
  if (o.scheme != FFTH_BASIC) {
    // r0 = b - A b = LS(x) - x
    const int fin_op = o.scheme == FFTH_CG ? FIN_RESID_INIT : FIN_BI_INIT;
    if ((s = apply<T>(P, d, nl, XF_LS, OP_GAMMA, XI_RESID, fin_op)) != FFTH_OK) return s;
  }
  if ((s = read_states(P)) != FFTH_OK) return s;
  int it = 0;
  while (it < o.max_iter && any_active(P, 0, nl)) {
    const int k = std::min(o.check_every, o.max_iter - it);
    if ((as = active_set(P, R_MAIN, 0, nl, 0)).n < 0) return FFTH_ERR_DEVICE;
    for (int j = 0; j < k; ++j) {
      if (o.scheme == FFTH_BASIC) s = apply<T>(P, as.d, as.n, XF_LS, OP_GAMMA, XI_BS, FIN_BS);
      else if (o.scheme == FFTH_CG) s = apply<T>(P, as.d, as.n, XF_CG, OP_GAMMA, XI_CG, FIN_CG_BETA);
      else s = bicg_iter<T>(P, as.d, as.n);
      if (s != FFTH_OK) return s;
    }
    it += k;
    if ((s = read_states(P)) != FFTH_OK) return s;
  }
  if (o.scheme == FFTH_BICGSTAB) {   // the last iteration's x update of every load
    ProfScope ps(P, C_POINT, nl);
    HIPCHK(Launch<T>::bicg_finish(dim3(ms_blocks(P->nvox), nl), P->stream, d, 6L * P->nvox));
  }
  return FFTH_OK;
}

// Three-term CG from x_0 = 0 (scheme FFTH_CG3): b = -Gamma0 * P_rhs into the
// residual slot (r_0 = b; the zero right-hand-side guard and ||b|| from its
// sums), the start pass, then fused iterations until the recursive residual
// meets the tolerance.  The last x ends in slot f(0) (formed by the finish
// kernel when the last iteration was even); FP64 copies it to the output,
// FP32 widens it in the common finish.
template <typename T> ffth_status run_cg3(ffth_plan* P, int nl) {
  const ffth_opts& o = P->opts;
  ffth_status s;
  DescSet as;
  if ((s = apply<T>(P, dptr(P, R_MAIN_DELTA), nl, XF_LS, OP_GAMMA, XI_BS, FIN_LS_FIRST)) != FFTH_OK) return s;
  if ((s = read_states(P)) != FFTH_OK) return s;
  if ((as = active_set(P, R_MAIN, 0, nl, 0)).n < 0) return FFTH_ERR_DEVICE;
  if ((s = cg3_start<T>(P, as.d, as.n, false)) != FFTH_OK) return s;
  if ((s = read_states(P)) != FFTH_OK) return s;
  int it = 0;
  while (it < o.max_iter && any_active(P, 0, nl)) {
    const int k = std::min(o.check_every, o.max_iter - it);
    if ((as = active_set(P, R_MAIN, 0, nl, 0)).n < 0) return FFTH_ERR_DEVICE;
    for (int j = 0; j < k; ++j)
      if ((s = cg3_iter<T>(P, as.d, as.n, false)) != FFTH_OK) return s;
    it += k;
    if ((s = read_states(P)) != FFTH_OK) return s;
  }
  // the last x of solves that stopped after an even iteration
  {
    ProfScope ps(P, C_POINT, nl);
    HIPCHK(Launch<T>::cg3_finish(dim3(ms_blocks(P->nvox), nl), P->stream, dptr(P, R_MAIN), 6L * P->nvox));
  }
  const size_t bytes = (size_t)P->nvox * 6 * sizeof(T);
  if (sizeof(T) == 8) {   // FP64: x_k ends in slot 0, copied to the output
    for (int l = 0; l < nl; ++l) {
      const Desc& m = P->h_desc[desc_slot(P, R_MAIN, l)];
      double* eps = (double*)P->h_desc[desc_slot(P, R_POST, l)].x;
      if (P->h_state[l].flag == FLAG_ZERO_RHS) HIPCHK(hipMemsetAsync(eps, 0, bytes, P->stream));
      else HIPCHK(hipMemcpyAsync(eps, m.x, bytes, hipMemcpyDeviceToDevice, P->stream));
    }
  }
  return FFTH_OK;
}

// ---- FP32 inner solves under an FP64 defect-correction loop -----------------
//
// A solve is a job stepping through phases.  One round advances every job of
// a group (same grid and material kind) by one phase step, with the loads of
// all jobs in the same phase sharing each launch:
//   A0    first FP64 residual sweep (x = 0, r = b, compatible): straight to INNER
//   A     FP64 residual sweep with x += delta fused, then PROJ
//   PROJ  split r with P = Gamma0 C0: compatible part -> FP32 inner right-hand
//         side, the rest (minus the incompatible round-off of x) applied to x
//   INNER up to check_every FP32 CG / Basic Scheme iterations
// Outer states sit in slots [0, nl), inner states in [nl, 2nl) of each plan.
enum Phase { PH_A0 = 0, PH_A, PH_PROJ, PH_INNER, PH_DONE };

struct Job {
  ffth_plan* P = nullptr;
  int nl = 0;
  int phase = PH_A0;
  int sweeps = 0;       // FP64 residual sweeps done
  int inner_total = 0;  // FP32 inner iterations launched (budget: opts.max_iter)
  bool last = false;    // inner budget spent: the next sweep is the final one
  bool fresh = false;   // inner solve entered: its three-term CG start pass is due
};

// Staging for the combined descriptor arrays of one round: a device array and
// its pinned host copy of `cap` descriptors, filled from `cursor` on.  Each
// job is in one phase per round, so a round stages each load at most twice
// (the sweep of a load whose inner solve owes its last x also stages that
// finish); the host copy is not rewritten before the streams the round's
// uploads were queued on have drained.
struct Stage {
  Desc* d;
  Desc* h;
  int cap;
  int cursor;
  bool overflow = false;   // an append found the area full (the round is refused)
};

// Append the descriptors of role r of job J whose state (slot base + l) was
// active at the last read-back.
int stage_append(Stage& st, const Job& J, Role r, int base) {
  int k = 0;
  for (int l = 0; l < J.nl; ++l)
    if (J.P->h_state[base + l].active) {
      if (st.cursor >= st.cap) {
        st.overflow = true;
        break;
      }
      st.h[st.cursor++] = J.P->h_desc[desc_slot(J.P, r, l)];
      ++k;
    }
  return k;
}

ffth_status stage_upload(hipStream_t stream, Stage& st, int from, int count, const Desc** out) {
  *out = st.d + from;
  if (count > 0)
    HIPCHK(hipMemcpyAsync(st.d + from, st.h + from, count * sizeof(Desc), hipMemcpyHostToDevice, stream));
  return FFTH_OK;
}

ffth_status enter_inner(Job& J) {
  ffth_plan* P = J.P;
  const size_t bytes = (size_t)P->nvox * 6 * sizeof(float);
  if (P->opts.scheme == FFTH_CG) {
    J.fresh = true;   // x_0 = 0 is implicit in the three-term CG
  } else {
    for (int l = 0; l < J.nl; ++l)   // Basic Scheme: x_0 = b
      HIPCHK(hipMemcpyAsync(f32_ptr(P, l, 0), f32_ptr(P, l, 1), bytes, hipMemcpyDeviceToDevice, P->stream));
  }
  J.phase = PH_INNER;
  return FFTH_OK;
}

// Inner iterations that a round leaves to a multi-size launch (three-term CG
// inner solves of a grid in the multi-size set): the staged range of the
// group's inner descriptors and the iterations the group asks for.
struct InnerSet {
  bool deferred = false;
  int from = 0, cnt = 0, kin = 0;
};

// Queue one round for a group of mixed-precision jobs sharing grid size,
// material kind, scheme and spectrum precision, on the first job's stream:
// the launches of every phase and the state read-back of every job.  Nothing
// waits for the device; group_advance runs once the stream has drained.
// *kin receives the inner iterations queued.  With defer set (and a grid of
// the multi-size set), the inner iterations and the read-backs of the jobs in
// the inner phase are left to the caller (*defer says which loads), who
// queues them on the same stream.
ffth_status group_issue(std::vector<Job*>& jobs, Stage& st, int* kin_out, InnerSet* defer = nullptr) {
  *kin_out = 0;
  if (jobs.empty()) return FFTH_OK;
  ffth_plan* dims = jobs[0]->P;
  const ffth_opts& o = dims->opts;
  ffth_status s;
  for (Job* J : jobs) {
    // one launch serves every job, with the first job's kernels: a binary16
    // kernel needs the FP32 copy (spec2) that only binary16 descriptors carry.
    // Tile shapes come from the first job's plan too; every plan's partial
    // sums are sized for the largest block count of any shape, and plans of
    // one grid, material kind, precision and scheme share the tuned shapes.
    const ffth_plan* P = J->P;
    if (P->n[0] != dims->n[0] || P->n[1] != dims->n[1] || P->n[2] != dims->n[2] || P->iso != dims->iso ||
        P->h16 != dims->h16 || P->opts.scheme != o.scheme || P->stream != dims->stream) {
      g_last_error = "jobs of one round differ in grid, material kind, scheme, spectrum precision or stream";
      return FFTH_ERR_INVALID;
    }
  }
  int from[4], cnt[4] = {0, 0, 0, 0}, nFresh = 0;
  int kin = o.check_every;
  const Role role[3] = {R_MAIN, R_MAIN_DELTA, R_PROJ};
  for (int ph = PH_A0; ph <= PH_PROJ; ++ph) {
    from[ph] = st.cursor;
    for (Job* J : jobs)
      if (J->phase == ph) cnt[ph] += stage_append(st, *J, role[ph], 0);
  }
  // the first sweep of a solve runs on the zero iterate: its passes skip reading it
  for (int i = 0; i < cnt[PH_A0]; ++i) st.h[from[PH_A0] + i].x_zero = 1;
  // inner loads: those whose solve starts this round first (they take the start pass)
  from[3] = st.cursor;
  for (int pass = 0; pass < 2; ++pass) {
    for (Job* J : jobs) {
      if (J->phase != PH_INNER || J->fresh != (pass == 0)) continue;
      cnt[3] += stage_append(st, *J, R_INNER, J->nl);
      if (pass == 0) nFresh = cnt[3];
      kin = std::min(kin, std::max(1, o.max_iter - J->inner_total));
    }
  }
  if (st.overflow) {
    st.overflow = false;
    g_last_error = "descriptor staging area too small for the round";
    return FFTH_ERR_INVALID;
  }
  // binary16 kernels read the operator output through spec2: every inner
  // descriptor must match the launch's spectrum precision
  if (!h16_launch_ok(st.h + from[3], cnt[3], dims->h16)) {
    g_last_error = "inner-solve descriptors do not match the launch's spectrum precision";
    return FFTH_ERR_INVALID;
  }
  // inner solves that ended after an even iteration owe their last x, which
  // the sweep of this round adds: formed first (once: the host launches it
  // in the round after the solve stopped, the only sweep round that follows)
  const int fromF = st.cursor;
  int cntF = 0;
  if (o.scheme == FFTH_CG) {
    for (Job* J : jobs) {
      if (J->phase != PH_A) continue;
      for (int l = 0; l < J->nl; ++l)
        if (J->P->h_state[J->nl + l].xpend) {
          if (st.cursor >= st.cap) {
            g_last_error = "descriptor staging area too small for the round";
            return FFTH_ERR_INVALID;
          }
          st.h[st.cursor++] = J->P->h_desc[desc_slot(J->P, R_INNER, l)];
          ++cntF;
        }
    }
  }
  hipStream_t sm = dims->stream;
  const Desc* d;
  // inner loads first: their descriptors and the start pass of fresh solves
  const Desc* din;
  if ((s = stage_upload(sm, st, from[3], cnt[3], &din)) != FFTH_OK) return s;
  const int nIN = cnt[3];
  if (o.scheme == FFTH_CG && (s = cg3_start<float>(dims, din, nFresh, dims->h16)) != FFTH_OK) return s;
  const bool deferred = defer && o.scheme == FFTH_CG && multi_grid(dims->n);
  if (deferred) *defer = InnerSet{true, from[3], nIN, kin};
  if ((s = stage_upload(sm, st, fromF, cntF, &d)) != FFTH_OK) return s;
  if (cntF > 0) {
    ProfScope ps(dims, C_POINT, cntF);
    HIPCHK(Launch<float>::cg3_finish(dim3(ms_blocks(dims->nvox), cntF), sm, d, 6L * dims->nvox));
  }
  if ((s = stage_upload(sm, st, from[0], cnt[0], &d)) != FFTH_OK) return s;
  if ((s = apply<double>(dims, d, cnt[0], XF_LS, OP_GAMMA, XI_RESID, FIN_OUTER)) != FFTH_OK) return s;
  if ((s = stage_upload(sm, st, from[1], cnt[1], &d)) != FFTH_OK) return s;
  if ((s = apply<double>(dims, d, cnt[1], XF_LS, OP_GAMMA, XI_RESID, FIN_OUTER_P)) != FFTH_OK) return s;
  if ((s = stage_upload(sm, st, from[2], cnt[2], &d)) != FFTH_OK) return s;
  if ((s = apply<float>(dims, d, cnt[2], XF_C0, OP_GAMMA, XI_PROJ, FIN_PROJ)) != FFTH_OK) return s;
  if (deferred) {
    for (Job* J : jobs) J->fresh = false;
    for (Job* J : jobs)
      if (J->phase != PH_INNER)
        HIPCHK(hipMemcpyAsync(J->P->h_state, J->P->d_state, J->P->L.nstate * sizeof(SolverState),
                              hipMemcpyDeviceToHost, sm));
    *kin_out = kin;
    return FFTH_OK;
  }
  for (int j = 0; j < kin && nIN > 0; ++j) {
    if (o.scheme == FFTH_BASIC) s = apply<float>(dims, din, nIN, XF_MATVEC, OP_GAMMA, XI_BS_INNER, FIN_BS);
    else s = cg3_iter<float>(dims, din, nIN, dims->h16);
    if (s != FFTH_OK) return s;
  }
  for (Job* J : jobs) J->fresh = false;
  for (Job* J : jobs)
    HIPCHK(hipMemcpyAsync(J->P->h_state, J->P->d_state, J->P->L.nstate * sizeof(SolverState),
                          hipMemcpyDeviceToHost, sm));
  *kin_out = kin;
  return FFTH_OK;
}

// Phase transitions of a group after its stream has drained (the states read
// back by group_issue are current).
ffth_status group_advance(std::vector<Job*>& jobs, int kin) {
  ffth_status s;
  for (Job* J : jobs) prof_flush(J->P);
  for (Job* J : jobs) {
    ffth_plan* P = J->P;
    const ffth_opts& o = P->opts;
    switch (J->phase) {
      case PH_A0:
      case PH_A:
        J->sweeps++;
        if (!any_active(P, 0, J->nl) || J->last || J->sweeps >= o.max_outer) J->phase = PH_DONE;
        else if (J->phase == PH_A0) {
          if ((s = enter_inner(*J)) != FFTH_OK) return s;
        } else J->phase = PH_PROJ;
        break;
      case PH_PROJ:
        if ((s = enter_inner(*J)) != FFTH_OK) return s;
        break;
      case PH_INNER:
        J->inner_total += kin;
        if (J->inner_total >= o.max_iter) J->last = true;
        if (!any_active(P, J->nl, J->nl) || J->last) J->phase = PH_A;
        break;
    }
  }
  return FFTH_OK;
}

ffth_status run_mixed(ffth_plan* P, int nl) {
  Job J;
  J.P = P;
  J.nl = nl;
  std::vector<Job*> jobs{&J};
  ffth_status s;
  while (J.phase != PH_DONE) {
    Stage st{P->d_cdesc, P->h_cdesc, 4 * P->nloads, 0};
    int kin = 0;
    if ((s = group_issue(jobs, st, &kin)) != FFTH_OK) return s;
    HIPCHK(hipStreamSynchronize(P->stream));
    if ((s = group_advance(jobs, kin)) != FFTH_OK) return s;
  }
  return FFTH_OK;
}

ffth_status check_plan(ffth_plan* P, int nloads) {
  if (!P) {
    g_last_error = "null plan";
    return FFTH_ERR_INVALID;
  }
  if (nloads < 1 || nloads > P->nloads) {
    g_last_error = "nloads outside [1, plan nloads]";
    return FFTH_ERR_INVALID;
  }
  return FFTH_OK;
}

// Fill descriptors of roles MAIN/MAIN_DELTA/INNER/POST for nl loads.
void build_solve_descs(ffth_plan* P, int nl, const double* E, double* eps, bool order1) {
  const ffth_opts& o = P->opts;
  for (int l = 0; l < nl; ++l) {
    Desc m = base_desc(P, l);
    if (E) {
      const double* e = E + 6 * l;
      for (int c = 0; c < 6; ++c) m.E[c] = c < 3 ? e[c] : 0.5 * e[c];
    }
    m.P = order1 ? Pfield(P, l) : nullptr;
    m.st = st_main(P, l);
    m.st2 = st_inner(P, l);
    double* epsl = eps + (size_t)l * 6 * P->nvox;
    if (o.scheme == FFTH_CG3) {
      // x_k, r_k in slots 0, 1 (k even) or 2, 3 (k odd) of the workspace
      if (o.precision == FFTH_FP64) {
        m.x = f64_ptr(P, l, 0);
        m.r = f64_ptr(P, l, 1);
        m.x1 = f64_ptr(P, l, 2);
        m.r1 = f64_ptr(P, l, 3);
      } else {
        m.x = f32_ptr(P, l, 0);
        m.r = f32_ptr(P, l, 1);
        m.x1 = f32_ptr(P, l, 2);
        m.r1 = f32_ptr(P, l, 3);
      }
    } else if (o.precision == FFTH_FP64) {
      m.x = epsl;
      if (o.scheme == FFTH_CG) {
        m.r = f64_ptr(P, l, 0);
        m.p = f64_ptr(P, l, 1);
      } else if (o.scheme == FFTH_BICGSTAB) {
        m.r = f64_ptr(P, l, 0);
        m.rh = f64_ptr(P, l, 1);
        m.p = f64_ptr(P, l, 2);
        m.v = f64_ptr(P, l, 3);
        m.s = f64_ptr(P, l, 4);
        m.t = f64_ptr(P, l, 5);
      }
    } else if (o.precision == FFTH_FP32) {
      m.x = f32_ptr(P, l, 0);
      if (o.scheme == FFTH_CG) {
        m.r = f32_ptr(P, l, 1);
        m.p = f32_ptr(P, l, 2);
      } else if (o.scheme == FFTH_BICGSTAB) {
        m.r = f32_ptr(P, l, 1);
        m.rh = f32_ptr(P, l, 2);
        m.p = f32_ptr(P, l, 3);
        m.v = f32_ptr(P, l, 4);
        m.s = f32_ptr(P, l, 5);
        m.t = f32_ptr(P, l, 6);
      }
    } else {  // MIXED: outer FP64 pass
      m.x = epsl;
      m.r = f32_ptr(P, l, 1);
      m.r_f32 = 1;
    }
    P->h_desc[desc_slot(P, R_MAIN, l)] = m;
    Desc md = m;
    Desc pr = m;
    if (o.precision == FFTH_MIXED) {
      // later sweeps: x += delta fused; full FP64 residual kept for its projection
      md.delta = f32_ptr(P, l, 0);
      md.delta_gate = o.scheme == FFTH_CG ? 1 : 0;
      md.r = f64_ptr(P, l, 0);
      md.r_f32 = 0;
      pr.r = f64_ptr(P, l, 0);
      pr.out = f32_ptr(P, l, 1);
    }
    if (o.scheme == FFTH_CG3) md.x = m.r;   // b = -Gamma0 * P_rhs goes to the residual slot (r_0 = b)
    P->h_desc[desc_slot(P, R_MAIN_DELTA, l)] = md;
    P->h_desc[desc_slot(P, R_PROJ, l)] = pr;
    Desc in = base_desc(P, l);
    in.st = st_inner(P, l);
    if (o.precision == FFTH_MIXED) {
      in.x = f32_ptr(P, l, 0);   // delta (slot 0)
      in.r = f32_ptr(P, l, 1);   // inner residual / right-hand side (slot 0)
      if (o.scheme == FFTH_CG) {
        in.x1 = f32_ptr(P, l, 2);
        in.r1 = f32_ptr(P, l, 3);
      }
      if (P->h16) set_h16(P, in);
    }
    P->h_desc[desc_slot(P, R_INNER, l)] = in;
    Desc post = base_desc(P, l);
    post.st = st_post(P, l);
    post.x = epsl;
    for (int c = 0; c < 6; ++c) post.E[c] = m.E[c];
    post.P = m.P;
    if (o.precision == FFTH_FP32) {
      post.x = f32_ptr(P, l, 0);  // widened into eps first (k_widen reads x, writes out)
      post.out = epsl;
    }
    P->h_desc[desc_slot(P, R_POST, l)] = post;
  }
}

// Run the solve for nl loads whose descriptors are built, then fill results.
// Upload the iteration states and zero the iterate of nl loads whose
// descriptors are built (keep_gscale: order-1 guard scales from the builder).
ffth_status solve_begin(ffth_plan* P, int nl, bool keep_gscale) {
  const ffth_opts& o = P->opts;
  ffth_status s;
  const double guard = o.precision == FFTH_FP32 ? 1e-6 : 1e-14;
  std::vector<SolverState> sts(3 * P->nloads + 1);
  for (int l = 0; l < P->nloads; ++l) {
    sts[l] = make_state(o.tol, o.precision == FFTH_MIXED ? o.max_outer : o.max_iter, guard, l < nl);
    sts[P->nloads + l] = make_state(o.inner_tol, o.max_iter, 1e-6, 0);
    sts[2 * P->nloads + l] = make_state(0, 1, 0, 1);
  }
  sts[3 * P->nloads] = make_state(0, 1, 0, 1);
  // keep the order-1 guard scales computed by the right-hand-side builder
  if (keep_gscale) {
    if ((s = read_states(P)) != FFTH_OK) return s;
    for (int l = 0; l < nl; ++l) sts[l].gscale = P->h_state[2 * P->nloads + l].gscale;
  }
  if ((s = upload_states(P, sts, 0)) != FFTH_OK) return s;
  // zero the iterate (three-term CG: the residual slot, which the first pass
  // reads as its iterate and overwrites with b)
  for (int l = 0; l < nl; ++l) {
    const Desc& m = P->h_desc[desc_slot(P, o.scheme == FFTH_CG3 ? R_MAIN_DELTA : R_MAIN, l)];
    const size_t bytes = (size_t)P->nvox * 6 * (o.precision == FFTH_FP32 ? sizeof(float) : sizeof(double));
    HIPCHK(hipMemsetAsync(m.x, 0, bytes, P->stream));
  }
  return FFTH_OK;
}

// After the iteration: exact zero for guarded loads, volume averages, results.
ffth_status solve_finish(ffth_plan* P, int nl, double* eps, ffth_result* res, double t0, const double* gmean) {
  const ffth_opts& o = P->opts;
  ffth_status s;
  // zero-rhs guard: eps = 0 exactly
  if ((s = read_states(P)) != FFTH_OK) return s;
  for (int l = 0; l < nl; ++l)
    if (P->h_state[l].flag == FLAG_ZERO_RHS) {
      const Desc& m = P->h_desc[desc_slot(P, R_MAIN, l)];
      const size_t bytes = (size_t)P->nvox * 6 * (o.precision == FFTH_FP32 ? sizeof(float) : sizeof(double));
      HIPCHK(hipMemsetAsync(m.x, 0, bytes, P->stream));
    }
  const Desc* dp = dptr(P, R_POST);
  if (o.precision == FFTH_FP32) {
    ProfScope ps(P, C_POINT, nl);
    HIPCHK(launch_widen(nl, P->stream, dp, (long)P->nvox * 6));
  }
  // mean stress: the post descriptors read eps (FP64)
  if (o.precision == FFTH_FP32) {
    for (int l = 0; l < nl; ++l) P->h_desc[desc_slot(P, R_POST, l)].x = eps + (size_t)l * 6 * P->nvox;
    if ((s = upload_descs(P)) != FFTH_OK) return s;
  }
  const int nms = ms_blocks(P->nvox);
  {
    ProfScope ps(P, C_POINT, nl);
    HIPCHK(launch_mean_stress(P->iso, nms, nl, P->stream, dp, P->nvox));
  }
  if ((s = fin(P, dp, nl, FIN_SUMS_I, 0, nms)) != FFTH_OK) return s;
  if ((s = read_states(P)) != FFTH_OK) return s;
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count() - t0;
  ffth_status worst = FFTH_OK;
  for (int l = 0; l < nl; ++l) {
    const SolverState& m = P->h_state[l];
    const SolverState& in = P->h_state[P->nloads + l];
    const SolverState& po = P->h_state[2 * P->nloads + l];
    ffth_result& r = res[l];
    std::memset(&r, 0, sizeof(r));
    if (m.flag == FLAG_CONVERGED || m.flag == FLAG_ZERO_RHS) r.status = FFTH_OK;
    else if (m.flag == FLAG_DIVERGED) r.status = FFTH_ERR_DIVERGED;
    else r.status = FFTH_ERR_NOT_CONVERGED;
    if (o.precision == FFTH_MIXED) {
      r.iters = in.total;
      r.outer_iters = m.iters;
      r.fp64_applications = m.fp64_apps;
      r.projections = m.proj;
    } else {
      r.iters = m.iters;
      // right-hand side (+ CG: r_0 = b - A b) and one application per iteration
      // (BiCGSTAB: two)
      const int apps = o.scheme == FFTH_BICGSTAB ? 2 * m.iters + 2 : m.iters + (o.scheme == FFTH_CG ? 2 : 1);
      r.fp64_applications = o.precision == FFTH_FP64 ? apps : 0;
    }
    r.residual = m.res;
    for (int c = 0; c < 6; ++c) r.mean_stress[c] = po.sums[c] / (double)P->nvox;
    if (gmean)
      for (int c = 0; c < 3; ++c) r.g_mean[c] = gmean[3 * l + c];
    r.seconds = secs;
    if (r.status != FFTH_OK && worst == FFTH_OK) worst = (ffth_status)r.status;
  }
  return worst;
}

ffth_status solve_common(ffth_plan* P, int nl, double* eps, ffth_result* res, double t0, const double* gmean) {
  ffth_status s;
  if ((s = solve_begin(P, nl, gmean != nullptr)) != FFTH_OK) return s;
  if (P->opts.precision == FFTH_FP64) s = run_plain<double>(P, dptr(P, R_MAIN), nl);
  else if (P->opts.precision == FFTH_FP32) s = run_plain<float>(P, dptr(P, R_MAIN), nl);
  else s = run_mixed(P, nl);
  if (s != FFTH_OK) return s;
  return solve_finish(P, nl, eps, res, t0, gmean);
}

double now_s() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
namespace {

void* host_get(ffth_plan* P, size_t bytes) {
  if (P->hpool) return P->hpool->get(bytes);
  void* q = nullptr;
  return hipHostMalloc(&q, bytes, hipHostMallocDefault) == hipSuccess ? q : nullptr;
}

void host_put(ffth_plan* P, void* q, size_t bytes) {
  if (!q) return;
  if (P->hpool) P->hpool->put(q, bytes);
  else (void)hipHostFree(q);
}

void free_host_bufs(ffth_plan* P) {
  host_put(P, P->h_state, P->L.nstate * sizeof(SolverState));
  host_put(P, P->h_cdesc, 4 * (size_t)P->nloads * sizeof(Desc));
  P->h_state = nullptr;
  P->h_cdesc = nullptr;
}

ffth_status plan_create(ffth_plan** out, const ffth_problem* p, const ffth_opts* o, int32_t nloads, int32_t order,
                        void* workspace, size_t bytes, void* hip_stream, HostPool* pool);

}  // namespace

extern "C" {

void ffth_default_opts(ffth_opts* o) {
  if (!o) return;
  o->scheme = FFTH_CG;
  o->precision = FFTH_MIXED;
  o->tol = 1e-8;
  o->max_iter = 20000;
  o->inner_tol = 1e-3;
  o->max_outer = 30;
  o->check_every = 8;
  o->autotune = 1;
  o->spectrum16 = 1;
}

int32_t ffth_size_supported(int32_t n) { return size_supported(n) ? 1 : 0; }

double ffth_stiffness_contrast(int32_t nphases, const double* lame, const double* stiffness) {
  if (nphases < 1 || (!lame && !stiffness)) return NAN;
  return stiffness_contrast(nphases, lame != nullptr, lame, stiffness);
}

size_t ffth_workspace_bytes(const int32_t n[3], int32_t nphases, int32_t nloads, int32_t order, const ffth_opts* o) {
  if (!n || !o || nloads < 1 || nphases < 1 || nphases > 65535 || order < 0 || order > 2) return 0;
  int nn[3] = {n[0], n[1], n[2]};
  if (!grid_supported(nn) || !opts_valid(*o)) return 0;
  return make_layout(nn, nphases, nloads, order, *o).total;
}

const char* ffth_status_string(ffth_status s) {
  switch (s) {
    case FFTH_OK: return "ok";
    case FFTH_ERR_INVALID: return "invalid argument";
    case FFTH_ERR_OOM: return "workspace too small";
    case FFTH_ERR_NOT_CONVERGED: return "not converged";
    case FFTH_ERR_DIVERGED: return "diverged";
    case FFTH_ERR_DEVICE: return "device error";
    case FFTH_ERR_BUSY: return "busy";
    case FFTH_ERR_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* ffth_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

ffth_status plan_create(ffth_plan** out, const ffth_problem* p, const ffth_opts* o, int32_t nloads, int32_t order,
                        void* workspace, size_t bytes, void* hip_stream, HostPool* pool) {
  g_last_error.clear();
  if (!out || !p || !o || !workspace) {
    g_last_error = "null argument";
    return FFTH_ERR_INVALID;
  }
  *out = nullptr;
  if (((uintptr_t)workspace) % ALIGN) {
    g_last_error = "workspace not 256-byte aligned";
    return FFTH_ERR_INVALID;
  }
  {
    int nn[3] = {p->n[0], p->n[1], p->n[2]};
    if (!grid_supported(nn)) {
      g_last_error = "unsupported grid " + std::to_string(nn[0]) + "x" + std::to_string(nn[1]) + "x" +
                     std::to_string(nn[2]);
      return FFTH_ERR_INVALID;
    }
  }
  if (p->nphases < 1 || p->nphases > 65535 || !p->phase || ((p->lame == nullptr) == (p->stiffness == nullptr))) {
    g_last_error = "bad phase table";
    return FFTH_ERR_INVALID;
  }
  if (!(p->mu0 != 0.0) || !(p->lambda0 + 2.0 * p->mu0 != 0.0) || !std::isfinite(p->mu0) ||
      !std::isfinite(p->lambda0)) {
    g_last_error = "reference medium needs mu0 != 0 and lambda0 + 2 mu0 != 0";
    return FFTH_ERR_INVALID;
  }
  if ((o->scheme == FFTH_CG || o->scheme == FFTH_CG3) && !(p->mu0 > 0.0 && 3.0 * p->lambda0 + 2.0 * p->mu0 > 0.0)) {
    g_last_error = "CG needs a positive definite reference medium";
    return FFTH_ERR_INVALID;
  }
  if (!opts_valid(*o) || nloads < 1 || order < 0 || order > 2) {
    g_last_error = "bad options";
    return FFTH_ERR_INVALID;
  }
  int nn[3] = {p->n[0], p->n[1], p->n[2]};
  Layout L = make_layout(nn, p->nphases, nloads, order, *o);
  if (bytes < L.total) {
    g_last_error = "workspace needs " + std::to_string(L.total) + " bytes";
    return FFTH_ERR_OOM;
  }
  ffth_plan* P = new ffth_plan();
  for (int d = 0; d < 3; ++d) P->n[d] = p->n[d];
  P->nvox = (long)p->n[0] * p->n[1] * p->n[2];
  P->h = p->n[2] / 2;
  P->rows = (long)p->n[0] * p->n[1];
  P->nph = p->nphases;
  P->iso = p->lame != nullptr;
  P->lam0 = p->lambda0;
  P->mu0 = p->mu0;
  P->phase = p->phase;
  P->stream = (hipStream_t)hip_stream;
  P->nloads = nloads;
  P->order = order;
  P->opts = *o;
  P->ws = (char*)workspace;
  P->L = L;
  P->mat64 = (double*)(P->ws + L.mat64);
  P->mat32 = (float*)(P->ws + L.mat32);
  P->d_desc = (Desc*)(P->ws + L.desc);
  P->d_state = (SolverState*)(P->ws + L.state);
  P->d_cdesc = (Desc*)(P->ws + L.cdesc);
  set_blocks(P);
  P->h_desc.assign(L.ndesc, Desc{});
  P->hpool = pool;
  P->h_state = (SolverState*)host_get(P, L.nstate * sizeof(SolverState));
  P->h_cdesc = (Desc*)host_get(P, 4 * (size_t)nloads * sizeof(Desc));
  if (!P->h_state || !P->h_cdesc) {
    g_last_error = "hipHostMalloc failed";
    free_host_bufs(P);
    delete P;
    return FFTH_ERR_DEVICE;
  }
  // material tables
  std::vector<double> m64((size_t)p->nphases * 72, 0.0);
  double m0[36];
  iso_to_m(p->lambda0, p->mu0, m0);
  for (int ph = 0; ph < p->nphases; ++ph) {
    if (P->iso) {
      const double lam = p->lame[2 * ph], mu = p->lame[2 * ph + 1];
      m64[ph * 4 + 0] = lam;
      m64[ph * 4 + 1] = mu;
      m64[ph * 4 + 2] = lam - p->lambda0;
      m64[ph * 4 + 3] = mu - p->mu0;
    } else {
      double m[36];
      voigt21_to_m(p->stiffness + 21 * ph, m);
      for (int i = 0; i < 36; ++i) {
        m64[ph * 72 + i] = m[i];
        m64[ph * 72 + 36 + i] = m[i] - m0[i];
      }
    }
  }
  std::vector<float> m32(m64.size());
  for (size_t i = 0; i < m64.size(); ++i) m32[i] = (float)m64[i];
  {
    double kmax = 0.0;
    for (int ph = 0; ph < p->nphases; ++ph) {
      if (P->iso) {
        kmax = std::max(kmax, 3.0 * std::fabs(m64[ph * 4 + 2]) + 2.0 * std::fabs(m64[ph * 4 + 3]));
      } else {
        for (int a = 0; a < 6; ++a) {
          double rs = 0.0;
          for (int b = 0; b < 6; ++b) rs += std::fabs(m64[ph * 72 + 36 + a * 6 + b]);
          kmax = std::max(kmax, rs);
        }
      }
    }
    P->kappa = std::max(kmax / std::fabs(p->mu0), 1e-3);
  }
  // binary16 rounding (unit 2^-11) times the stiffness contrast bounds the
  // relative error the stored spectrum adds to the inner solve's operator;
  // above FFTH_SPECTRUM16_MAX_CONTRAST it would cost iterations, so FP32 is
  // kept; below FFTH_SPECTRUM16_MIN_VOXELS the launches are latency-bound
  P->contrast = stiffness_contrast(p->nphases, P->iso, p->lame, p->stiffness);
  P->h16 = o->precision == FFTH_MIXED && o->scheme == FFTH_CG && o->spectrum16 != 0 &&
           P->contrast <= FFTH_SPECTRUM16_MAX_CONTRAST &&
           (o->spectrum16 == 2 || P->nvox >= FFTH_SPECTRUM16_MIN_VOXELS);
  // the binary16 spectrum and its FP32 copy share the load's spectrum region
  // (sized for FP64: 48 bytes per voxel)
  if (P->h16 && al((size_t)P->nvox * 12) + (size_t)P->nvox * 24 > L.spec_stride) P->h16 = false;
  bool ok = hip_ok(hipMemcpyAsync(P->mat64, m64.data(), m64.size() * 8, hipMemcpyHostToDevice, P->stream), "copy") &&
            hip_ok(hipMemcpyAsync(P->mat32, m32.data(), m32.size() * 4, hipMemcpyHostToDevice, P->stream), "copy");
  // phase ids must index the table
  int* dmax = (int*)(P->ws + L.misc);
  ok = ok && hip_ok(hipMemsetAsync(dmax, 0, sizeof(int), P->stream), "memset") &&
       hip_ok(launch_phase_max(P->stream, p->phase, P->nvox, dmax), "phase check");
  int hmax = 0;
  ok = ok && hip_ok(hipMemcpyAsync(&hmax, dmax, sizeof(int), hipMemcpyDeviceToHost, P->stream), "copy") &&
       hip_ok(hipStreamSynchronize(P->stream), "sync");
  if (!ok) {
    free_host_bufs(P);
    delete P;
    return FFTH_ERR_DEVICE;
  }
  if (hmax >= p->nphases) {
    g_last_error = "phase id " + std::to_string(hmax) + " >= nphases";
    free_host_bufs(P);
    delete P;
    return FFTH_ERR_INVALID;
  }
  ffth_status ts = autotune(P);
  if (ts != FFTH_OK) {
    free_host_bufs(P);
    delete P;
    return ts;
  }
  *out = P;
  return FFTH_OK;
}

}  // namespace

extern "C" {

ffth_status ffth_plan_create(ffth_plan** out, const ffth_problem* p, const ffth_opts* o, int32_t nloads, int32_t order,
                             void* workspace, size_t bytes, void* hip_stream) {
  return plan_create(out, p, o, nloads, order, workspace, bytes, hip_stream, nullptr);
}

ffth_status ffth_plan_destroy(ffth_plan* P) {
  if (!P) return FFTH_ERR_INVALID;
  (void)hipStreamSynchronize(P->stream);
  prof_flush(P);
  for (hipEvent_t e : P->pool) (void)hipEventDestroy(e);
  free_host_bufs(P);
  delete P;
  return FFTH_OK;
}

ffth_status ffth_solve_order0(ffth_plan* P, int32_t nloads, const double* E, double* eps, ffth_result* res) {
  g_last_error.clear();
  ffth_status s = check_plan(P, nloads);
  if (s != FFTH_OK) return s;
  if (!E || !eps || !res) {
    g_last_error = "null argument";
    return FFTH_ERR_INVALID;
  }
  const double t0 = now_s();
  build_solve_descs(P, nloads, E, eps, false);
  if ((s = upload_descs(P)) != FFTH_OK) return s;
  return solve_common(P, nloads, eps, res, t0, nullptr);
}

namespace {

// Order-1 polarization P_l = p_2 + theta_2 for nl gradient loads (X1 built).
// Right-hand side P = p + theta of order 1 (G: [nl][18], pointwise data eps0,
// X1) or order 2 (G: [nl][54] second gradients, pointwise data eps1, X1, X2).
ffth_status build_rhs(ffth_plan* P, int order, int nl, const double* eps, const double* G, double* const* Pout,
                      std::vector<double>& gmean) {
  ffth_status s;
  for (int l = 0; l < nl; ++l) {
    Desc d = base_desc(P, l);
    d.st = st_post(P, l);
    if (order == 1)
      for (int i = 0; i < 18; ++i) d.G[i] = G[18 * l + i];
    else
      for (int i = 0; i < 54; ++i) d.H[i] = G[54 * l + i];
    d.io = Pout[l];          // p_2 out (then theta accumulated)
    d.p = gfield(P, l);      // g out
    P->h_desc[desc_slot(P, R_POST, l)] = d;
    Desc t = base_desc(P, l);
    t.st = st_post(P, l);
    t.io = gfield(P, l);     // copy-in g (3 components)
    t.nc = 3;
    t.out = Pout[l];         // accumulate theta (6 components) into P
    t.nc_out = 6;
    P->h_desc[desc_slot(P, R_THETA, l)] = t;
  }
  if ((s = upload_descs(P)) != FFTH_OK) return s;
  std::vector<SolverState> post(nl, make_state(0, 1, 0, 1));
  if ((s = upload_states(P, post, 2 * P->nloads)) != FFTH_OK) return s;
  const int nms = ms_blocks(P->nvox);
  {
    ProfScope ps(P, C_POINT, nl);
    if (order == 1)
      HIPCHK(launch_order1_point(P->iso, nms, nl, P->stream, dptr(P, R_POST), eps, X1field(P), P->nvox));
    else
      HIPCHK(launch_order2_point(P->iso, nms, nl, P->stream, dptr(P, R_POST), eps, X1field(P), X2field(P),
                                 P->nvox));
  }
  if ((s = fin(P, dptr(P, R_POST), nl, FIN_O1RHS, 0, nms)) != FFTH_OK) return s;
  const Desc* dt = dptr(P, R_THETA);
  if ((s = xfwd<double>(P, dt, nl, XF_COPY)) != FFTH_OK) return s;
  if ((s = yzy<double>(P, dt, nl, OP_THETA)) != FFTH_OK) return s;
  if ((s = xinv<double>(P, dt, nl, XI_ACCUM)) != FFTH_OK) return s;
  if ((s = read_states(P)) != FFTH_OK) return s;
  gmean.assign(3 * nl, 0.0);
  for (int l = 0; l < nl; ++l)
    for (int c = 0; c < 3; ++c) gmean[3 * l + c] = P->h_state[2 * P->nloads + l].sums[2 + c] / (double)P->nvox;
  return FFTH_OK;
}

ffth_status make_x1_block(ffth_plan* P, const double* eps0, double* out, int count);

// Displacements of `count` strain fields [count][6][N] into out [count][3][N]
// (order-0 correctors -> X1, order-1 unit-gradient solutions -> X2).
ffth_status make_disp(ffth_plan* P, const double* eps0, double* out, int count) {
  ffth_status s;
  for (int base = 0; base < count; base += 6) {
    const int k = std::min(6, count - base);
    if ((s = make_x1_block(P, eps0 + (size_t)base * 6 * P->nvox, out + (size_t)base * 3 * P->nvox, k)) != FFTH_OK)
      return s;
  }
  return FFTH_OK;
}

ffth_status make_x1(ffth_plan* P, const double* eps0) { return make_disp(P, eps0, X1field(P), 6); }

ffth_status make_x1_block(ffth_plan* P, const double* eps0, double* out, int count) {
  // Displacement transforms (forward, displacement operator, inverse) of
  // `count` <= 6 strain fields: as many fields per launch as the plan has
  // load spectra (each field in its own spectrum region and partial sums),
  // all groups queued back to back without waiting for the device.
  ffth_status s;
  const int k = std::max(1, std::min(count, P->nloads));
  for (int J = 0; J < count; ++J) {
    const int l = J % k;
    Desc d = base_desc(P, l);
    d.st = P->d_state + 3 * P->nloads;
    d.io = (void*)(eps0 + (size_t)J * 6 * P->nvox);
    d.out = out + (size_t)J * 3 * P->nvox;
    d.nc = 6;
    d.nc_out = 3;
    P->h_desc[util6_slot(P, J)] = d;
  }
  if ((s = upload_descs(P)) != FFTH_OK) return s;
  std::vector<SolverState> u(1, make_state(0, 1, 0, 1));
  if ((s = upload_states(P, u, 3 * P->nloads)) != FFTH_OK) return s;
  for (int J0 = 0; J0 < count; J0 += k) {
    const int nb = std::min(k, count - J0);
    const Desc* d = P->d_desc + util6_slot(P, J0);
    if ((s = xfwd<double>(P, d, nb, XF_COPY)) != FFTH_OK) return s;
    if ((s = yzy<double>(P, d, nb, OP_DISP)) != FFTH_OK) return s;
    if ((s = xinv<double>(P, d, nb, XI_STORE)) != FFTH_OK) return s;
  }
  return FFTH_OK;
}

}  // namespace

ffth_status ffth_solve_order1(ffth_plan* P, const double* eps0_six, int32_t nloads, const double* G, double* eps,
                              ffth_result* res) {
  g_last_error.clear();
  ffth_status s = check_plan(P, nloads);
  if (s != FFTH_OK) return s;
  if (P->order != 1) {
    g_last_error = "plan was created for order 0";
    return FFTH_ERR_INVALID;
  }
  if (!eps0_six || !G || !eps || !res) {
    g_last_error = "null argument";
    return FFTH_ERR_INVALID;
  }
  const double t0 = now_s();
  if ((s = make_x1(P, eps0_six)) != FFTH_OK) return s;
  std::vector<double*> pout(nloads);
  for (int l = 0; l < nloads; ++l) pout[l] = Pfield(P, l);
  std::vector<double> gmean;
  if ((s = build_rhs(P, 1, nloads, eps0_six, G, pout.data(), gmean)) != FFTH_OK) return s;
  build_solve_descs(P, nloads, nullptr, eps, true);
  if ((s = upload_descs(P)) != FFTH_OK) return s;
  return solve_common(P, nloads, eps, res, t0, gmean.data());
}

ffth_status ffth_solve_order2(ffth_plan* P, const double* eps0_six, const double* eps1_18, int32_t nloads,
                              const double* H, double* eps, ffth_result* res) {
  g_last_error.clear();
  ffth_status s = check_plan(P, nloads);
  if (s != FFTH_OK) return s;
  if (P->order != 2) {
    g_last_error = "plan was not created for order 2";
    return FFTH_ERR_INVALID;
  }
  if (!eps0_six || !eps1_18 || !H || !eps || !res) {
    g_last_error = "null argument";
    return FFTH_ERR_INVALID;
  }
  const double t0 = now_s();
  if ((s = make_x1(P, eps0_six)) != FFTH_OK) return s;
  if ((s = make_disp(P, eps1_18, X2field(P), 18)) != FFTH_OK) return s;
  std::vector<double*> pout(nloads);
  for (int l = 0; l < nloads; ++l) pout[l] = Pfield(P, l);
  std::vector<double> gmean;
  if ((s = build_rhs(P, 2, nloads, eps1_18, H, pout.data(), gmean)) != FFTH_OK) return s;
  build_solve_descs(P, nloads, nullptr, eps, true);
  if ((s = upload_descs(P)) != FFTH_OK) return s;
  return solve_common(P, nloads, eps, res, t0, gmean.data());
}

ffth_status ffth_order2_rhs(ffth_plan* P, const double* eps0_six, const double* eps1_18, const double* H,
                            double* Pout, double* g_mean) {
  g_last_error.clear();
  ffth_status s = check_plan(P, 1);
  if (s != FFTH_OK) return s;
  if (P->order != 2) {
    g_last_error = "plan was not created for order 2";
    return FFTH_ERR_INVALID;
  }
  if (!eps0_six || !eps1_18 || !H || !Pout) {
    g_last_error = "null argument";
    return FFTH_ERR_INVALID;
  }
  if ((s = make_x1(P, eps0_six)) != FFTH_OK) return s;
  if ((s = make_disp(P, eps1_18, X2field(P), 18)) != FFTH_OK) return s;
  std::vector<double> gm;
  double* po[1] = {Pout};
  if ((s = build_rhs(P, 2, 1, eps1_18, H, po, gm)) != FFTH_OK) return s;
  if (g_mean)
    for (int c = 0; c < 3; ++c) g_mean[c] = gm[c];
  HIPCHK(hipStreamSynchronize(P->stream));
  return FFTH_OK;
}

ffth_status ffth_green_apply(ffth_plan* P, const double* tau, double* eta, int32_t precision) {
  g_last_error.clear();
  ffth_status s = check_plan(P, 1);
  if (s != FFTH_OK) return s;
  if (!tau || !eta || (precision != FFTH_FP64 && precision != FFTH_FP32)) {
    g_last_error = "bad argument";
    return FFTH_ERR_INVALID;
  }
  Desc d = base_desc(P, 0);
  d.st = P->d_state + 3 * P->nloads;
  d.io = (void*)tau;
  d.out = eta;
  d.nc = 6;
  P->h_desc[desc_slot(P, R_UTIL, 0)] = d;
  if ((s = upload_descs(P)) != FFTH_OK) return s;
  std::vector<SolverState> u(1, make_state(0, 1, 0, 1));
  if ((s = upload_states(P, u, 3 * P->nloads)) != FFTH_OK) return s;
  const Desc* dd = dptr(P, R_UTIL);
  if (precision == FFTH_FP64) {
    if ((s = xfwd<double>(P, dd, 1, XF_COPY)) != FFTH_OK) return s;
    if ((s = yzy<double>(P, dd, 1, OP_GAMMA)) != FFTH_OK) return s;
    if ((s = xinv<double>(P, dd, 1, XI_STORE)) != FFTH_OK) return s;
  } else {
    if ((s = xfwd<float>(P, dd, 1, XF_COPY)) != FFTH_OK) return s;
    if ((s = yzy<float>(P, dd, 1, OP_GAMMA)) != FFTH_OK) return s;
    if ((s = xinv<float>(P, dd, 1, XI_STORE)) != FFTH_OK) return s;
  }
  HIPCHK(hipStreamSynchronize(P->stream));
  return FFTH_OK;
}

ffth_status ffth_displacement(ffth_plan* P, const double* eps, double* u) {
  g_last_error.clear();
  ffth_status s = check_plan(P, 1);
  if (s != FFTH_OK) return s;
  if (!eps || !u) {
    g_last_error = "null argument";
    return FFTH_ERR_INVALID;
  }
  Desc d = base_desc(P, 0);
  d.st = P->d_state + 3 * P->nloads;
  d.io = (void*)eps;
  d.out = u;
  d.nc = 6;
  d.nc_out = 3;
  P->h_desc[desc_slot(P, R_UTIL, 0)] = d;
  if ((s = upload_descs(P)) != FFTH_OK) return s;
  std::vector<SolverState> st(1, make_state(0, 1, 0, 1));
  if ((s = upload_states(P, st, 3 * P->nloads)) != FFTH_OK) return s;
  const Desc* dd = dptr(P, R_UTIL);
  if ((s = xfwd<double>(P, dd, 1, XF_COPY)) != FFTH_OK) return s;
  if ((s = yzy<double>(P, dd, 1, OP_DISP)) != FFTH_OK) return s;
  if ((s = xinv<double>(P, dd, 1, XI_STORE)) != FFTH_OK) return s;
  HIPCHK(hipStreamSynchronize(P->stream));
  return FFTH_OK;
}

ffth_status ffth_order1_rhs(ffth_plan* P, const double* eps0_six, const double* G, double* Pout, double* g_mean) {
  g_last_error.clear();
  ffth_status s = check_plan(P, 1);
  if (s != FFTH_OK) return s;
  if (P->order != 1) {
    g_last_error = "plan was created for order 0";
    return FFTH_ERR_INVALID;
  }
  if (!eps0_six || !G || !Pout) {
    g_last_error = "null argument";
    return FFTH_ERR_INVALID;
  }
  if ((s = make_x1(P, eps0_six)) != FFTH_OK) return s;
  std::vector<double> gm;
  double* po[1] = {Pout};
  if ((s = build_rhs(P, 1, 1, eps0_six, G, po, gm)) != FFTH_OK) return s;
  if (g_mean)
    for (int c = 0; c < 3; ++c) g_mean[c] = gm[c];
  HIPCHK(hipStreamSynchronize(P->stream));
  return FFTH_OK;
}

ffth_status ffth_profile_enable(ffth_plan* P, int32_t on) {
  if (!P) return FFTH_ERR_INVALID;
  HIPCHK(hipStreamSynchronize(P->stream));
  prof_flush(P);
  for (int c = 0; c < NCAT; ++c) {
    P->prof_ms[c] = 0.0;
    P->prof_n[c] = 0;
    P->prof_units[c] = 0;
  }
  P->prof = on != 0;
  return FFTH_OK;
}

ffth_status ffth_profile_read(ffth_plan* P, int32_t category, int64_t* launches, int64_t* units, double* ms) {
  if (!P || category < 0 || category >= NCAT || !launches || !units || !ms) return FFTH_ERR_INVALID;
  HIPCHK(hipStreamSynchronize(P->stream));
  prof_flush(P);
  *launches = P->prof_n[category];
  *units = P->prof_units[category];
  *ms = P->prof_ms[category];
  return FFTH_OK;
}

ffth_status ffth_tile_variants(ffth_plan* P, int32_t out[8]) {
  if (!P || !out) return FFTH_ERR_INVALID;
  for (int i = 0; i < 8; ++i) out[i] = P->var[i / 2][i % 2];
  return FFTH_OK;
}

ffth_status ffth_set_tile_variants(ffth_plan* P, const int32_t in[8]) {
  g_last_error.clear();
  if (!P || !in) return FFTH_ERR_INVALID;
  for (int i = 0; i < 8; ++i) {
    if (in[i] < 0 || in[i] >= NVAR) {
      g_last_error = "tile variant out of range";
      return FFTH_ERR_INVALID;
    }
  }
  for (int i = 0; i < 8; ++i) P->var[i / 2][i % 2] = in[i];
  set_blocks(P);
  return FFTH_OK;
}

ffth_status ffth_launch_loads(ffth_plan* P, int32_t out[2]) {
  if (!P || !out) return FFTH_ERR_INVALID;
  out[0] = P->bw[0];
  out[1] = P->bw[1];
  return FFTH_OK;
}

ffth_status ffth_set_launch_loads(ffth_plan* P, const int32_t in[2]) {
  g_last_error.clear();
  if (!P || !in) return FFTH_ERR_INVALID;
  if (in[0] < 0 || in[1] < 0) {
    g_last_error = "loads per launch must be >= 0";
    return FFTH_ERR_INVALID;
  }
  P->bw[0] = in[0];
  P->bw[1] = in[1];
  return FFTH_OK;
}

const char* ffth_profile_name(int32_t category) {
  return (category >= 0 && category < NCAT) ? CAT_NAMES[category] : "";
}

}  // extern "C"

// ===========================================================================
// Serving: continuous batching of order-0 solves inside a caller-owned arena
// ===========================================================================
namespace {

struct Request {
  uint64_t id = 0;
  int nl = 0;
  int n[3] = {0, 0, 0};
  bool iso = true;
  ffth_problem prob{};
  std::vector<double> table;      // host copy of lame / stiffness
  std::vector<double> E;
  size_t off = 0, bytes = 0, ws_bytes = 0;
  bool placed = false;            // [off, off + bytes) of the arena belongs to this request
  ffth_plan* P = nullptr;
  double* eps = nullptr;
  Job job;
  int state = 0;                  // 0 waiting, 1 running, 2 done, 3 cancelled
  ffth_status status = FFTH_OK;
  std::vector<ffth_result> res;
  double t_submit = 0, t_start = 0;
  int bypassed = 0;               // admissions that passed this request while it waited
};

size_t request_bytes(const int n[3], int nph, int nl, const ffth_opts& o, size_t* ws) {
  int nn[3] = {n[0], n[1], n[2]};
  const size_t w = make_layout(nn, nph, nl, 0, o).total;
  if (ws) *ws = w;
  const size_t nvox = (size_t)n[0] * n[1] * n[2];
  return al(w) + al((size_t)nl * 6 * nvox * sizeof(double));
}

}  // namespace

// Streams of a server: the caller's and FFTH_SERVER_STREAMS - 1 of its own.
// Each grid size is bound to one of them (in order of first appearance), so
// the launches of different sizes queue on different hardware queues and run
// concurrently; one step waits for all of them once.
constexpr int FFTH_SERVER_STREAMS = 4;

struct ffth_server {
  char* arena = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  std::vector<hipStream_t> streams;         // [0] = the caller's; the rest created here
  // Admission (material upload, phase-id check, descriptors, states) runs on
  // a stream of its own, which no round uses, so that its synchronizations
  // wait for the admission's own copies only and never for a round in flight
  // on the request's stream; the request's plan then moves to that stream.
  hipStream_t admit_stream = nullptr;
  HostPool hpool;                           // pinned mirrors of the request plans
  std::map<std::array<int, 3>, int> size_stream;   // grid -> index into streams
  ffth_opts opts{};
  int max_running = 0;
  int max_bypass = 0;                      // admissions that may pass a waiting request
  int64_t multi_iterations = 0;            // inner iterations run as multi-size launches
  int32_t multi_max_grids = 0;             // most distinct grids in one multi-size launch
  // Each stream runs its own rounds: a round is issued on an idle stream, and
  // completed (phase transitions, finished requests) once its event has
  // passed, independently of the other streams.
  struct Round {
    bool busy = false;
    hipEvent_t done = nullptr;             // recorded after the round's last command
    std::vector<std::vector<Job*>> groups; // the round's launch groups
    std::vector<int> kin;                  // inner iterations each group ran
  };
  std::vector<Round> rounds;               // per stream
  std::vector<Stage> stages;               // descriptor staging per stream (a round's are in flight)
  size_t stage_bytes = 0;                  // arena bytes of all streams' staging areas
  FreeList free_;                          // free ranges of the arena
  std::deque<Request*> waiting;
  std::vector<Request*> running;
  std::map<uint64_t, Request*> reqs;
  uint64_t next = 1;
};

namespace {

void finish_request(ffth_server* S, Request* r, ffth_status st) {
  if (r->P) {
    (void)ffth_plan_destroy(r->P);
    r->P = nullptr;
  }
  // only memory the request was placed in goes back (a waiting request holds none)
  if (r->placed && !S->free_.release(r->off, r->bytes)) g_last_error = "arena bookkeeping: overlapping release refused";
  r->placed = false;
  r->status = st;
  r->state = st == FFTH_ERR_CANCELLED ? 3 : 2;
}

hipStream_t stream_for(ffth_server* S, const int n[3]) {
  const std::array<int, 3> key{n[0], n[1], n[2]};
  auto it = S->size_stream.find(key);
  if (it == S->size_stream.end())
    it = S->size_stream.emplace(key, (int)(S->size_stream.size() % S->streams.size())).first;
  return S->streams[it->second];
}

// Admit waiting requests while a slot is free: the request of least work
// (voxels x load cases) whose memory fits the free arena goes first, so that
// small requests do not queue behind a large head; a request passed over
// max_bypass times is admitted next, as soon as its memory fits, and nothing
// passes it meanwhile (admission.h).
ffth_status admit(ffth_server* S) {
  while (!S->waiting.empty() && (int)S->running.size() < S->max_running) {
    std::vector<WaitInfo> q;
    q.reserve(S->waiting.size());
    for (const Request* w : S->waiting)
      q.push_back({w->bytes, (double)w->n[0] * w->n[1] * w->n[2] * w->nl, w->bypassed});
    const int k = pick_next(q, S->free_, S->max_bypass);
    if (k < 0) break;
    Request* r = S->waiting[k];
    size_t off;
    if (!S->free_.alloc(r->bytes, &off)) break;
    for (int i = 0; i < k; ++i) S->waiting[i]->bypassed++;
    S->waiting.erase(S->waiting.begin() + k);
    if (off < S->stage_bytes || off + r->bytes > S->bytes) {   // never place over the staging areas
      finish_request(S, r, FFTH_ERR_OOM);
      continue;
    }
    r->off = off;
    r->placed = true;
    r->prob.lame = r->iso ? r->table.data() : nullptr;
    r->prob.stiffness = r->iso ? nullptr : r->table.data();
    // grids whose inner iterations run as multi-size launches keep the
    // default tiles (those launches use them), so that every pass of the
    // request is what the plan path computes with autotuning off
    ffth_opts po = S->opts;
    if (po.scheme == FFTH_CG && multi_grid(r->n)) po.autotune = 0;
    ffth_status st = plan_create(&r->P, &r->prob, &po, r->nl, 0, S->arena + off, r->ws_bytes, S->admit_stream,
                                 &S->hpool);
    if (st != FFTH_OK) {
      r->P = nullptr;
      finish_request(S, r, st);
      continue;
    }
    r->eps = (double*)(S->arena + off + al(r->ws_bytes));
    r->t_start = now_s();
    build_solve_descs(r->P, r->nl, r->E.data(), r->eps, false);
    if ((st = upload_descs(r->P)) != FFTH_OK || (st = solve_begin(r->P, r->nl, false)) != FFTH_OK ||
        (st = hip_ok(hipStreamSynchronize(S->admit_stream), "sync") ? FFTH_OK : FFTH_ERR_DEVICE) != FFTH_OK) {
      finish_request(S, r, st);
      continue;
    }
    // everything the admission queued has completed: the rounds take over
    r->P->stream = stream_for(S, r->n);
    r->job = Job();
    r->job.P = r->P;
    r->job.nl = r->nl;
    r->state = 1;
    S->running.push_back(r);
  }
  return FFTH_OK;
}


using GroupMap = std::map<std::tuple<int, int, int, bool, bool>, std::vector<Job*>>;

// The inner iterations the groups of a step deferred (grids of the
// multi-size set), as one launch per pass for every group of one size
// stream, material kind and spectrum precision, on that stream after the
// groups' rounds (grids share a stream when there are more of them than
// streams; their launches would run one after the other anyway, so merging
// them costs no concurrency and saves launches): the staged inner
// descriptors of those groups are copied into one array, each with the
// block count of its fused pass for the finalize.  Every group of a set runs
// the smallest of the iteration counts its groups asked for (kin updated);
// the states of their jobs in the inner phase are read back after the last
// iteration.
ffth_status issue_merged(ffth_server* S, Stage& stage, GroupMap& groups, const std::vector<InnerSet>& inner,
                         std::vector<int>& kin) {
  size_t g = 0;
  for (hipStream_t m : S->streams) {
    for (int iso = 0; iso < 2; ++iso) {
      for (int h16 = 0; h16 < 2; ++h16) {
        const int from = stage.cursor;
        int cnt = 0, kmin = INT32_MAX;
        struct Seg {
          int first, count, nb[3];
        };
        std::vector<Seg> segs;   // one per grid with inner loads, descriptors consecutive from `from`
        std::vector<size_t> members;
        g = 0;
        for (auto& kv : groups) {
          const InnerSet& is = inner[g];
          const ffth_plan* P0 = kv.second[0]->P;
          if (is.deferred && P0->stream == m && P0->iso == (iso != 0) && P0->h16 == (h16 != 0)) {
            members.push_back(g);
            kmin = std::min(kmin, is.kin);
            if (stage.cursor + is.cnt > stage.cap) {
              g_last_error = "descriptor staging area too small for the step";
              return FFTH_ERR_INVALID;
            }
            Seg sg{cnt, is.cnt, {0, 0, 0}};
            multi_blocks(P0->n, sg.nb);
            for (int i = 0; i < is.cnt; ++i) {
              Desc dd = stage.h[is.from + i];
              dd.nblk_multi = sg.nb[2];
              stage.h[stage.cursor++] = dd;
            }
            if (is.cnt > 0) {
              segs.push_back(sg);
              cnt += is.cnt;
            }
          }
          ++g;
        }
        if (members.empty()) continue;
        if (cnt > 0) {
          if (!h16_launch_ok(stage.h + from, cnt, h16 != 0)) {
            g_last_error = "inner-solve descriptors do not match the launch's spectrum precision";
            return FFTH_ERR_INVALID;
          }
          const Desc* d;
          ffth_status s;
          if ((s = stage_upload(m, stage, from, cnt, &d)) != FFTH_OK) return s;
          // segment tables per pass, MULTI_SEGS grids per launch; each load's
          // blocks are padded to a multiple of the 8 XCDs
          std::vector<std::array<MultiSegs, 3>> tabs;
          for (size_t c0 = 0; c0 < segs.size(); c0 += MULTI_SEGS) {
            std::array<MultiSegs, 3> t;
            for (int pass = 0; pass < 3; ++pass) {
              MultiSegs& ms = t[pass];
              std::memset(&ms, 0, sizeof(ms));
              for (size_t c = c0; c < segs.size() && c < c0 + MULTI_SEGS; ++c) {
                const int k = ms.n++;
                ms.first[k] = segs[c].first;
                ms.bpd[k] = segs[c].nb[pass];
                ms.off[k + 1] = ms.off[k] + segs[c].count * ((segs[c].nb[pass] + 7) / 8 * 8);
              }
            }
            tabs.push_back(t);
          }
          for (int j = 0; j < kmin; ++j) {
            for (auto& t : tabs) HIPCHK(multi_ypass(t[0], m, d, -1, h16 != 0));
            for (auto& t : tabs) HIPCHK(multi_zpass(t[1], m, d, OP_GAMMA, h16 != 0));
            // the inverse y-transform reads the FP32 copy of a binary16 inner solve
            for (auto& t : tabs) HIPCHK(multi_ypass(t[0], m, d, +1, false));
            for (auto& t : tabs) HIPCHK(multi_xcg3(t[2], m, d, iso != 0, h16 != 0));
            HIPCHK(launch_finalize(cnt, m, d, FIN_CG3, 0, -1));
          }
          S->multi_iterations += kmin;
          S->multi_max_grids = std::max(S->multi_max_grids, (int32_t)std::min<size_t>(segs.size(), MULTI_SEGS));
        }
        for (size_t gm : members) kin[gm] = kmin;
        g = 0;
        for (auto& kv : groups) {
          if (std::find(members.begin(), members.end(), g++) == members.end()) continue;
          for (Job* J : kv.second)
            if (J->phase == PH_INNER)
              HIPCHK(hipMemcpyAsync(J->P->h_state, J->P->d_state, J->P->L.nstate * sizeof(SolverState),
                                    hipMemcpyDeviceToHost, m));
        }
      }
    }
  }
  return FFTH_OK;
}

// Issue the next round of stream k: every running request bound to it,
// grouped by grid, material kind and spectrum precision (a group's launches
// take its first job's kernels); the inner iterations of multi-size grids
// that share the stream are deferred and run together, one launch per pass
// across their sizes (issue_merged).  A group joins such a launch only when
// another group with inner iterations in this round shares its material kind
// and spectrum precision (a grid alone on the stream keeps the per-size
// kernels, whose default tiles compute the same values).
ffth_status issue_round(ffth_server* S, size_t k) {
  ffth_server::Round& R = S->rounds[k];
  hipStream_t sm = S->streams[k];
  GroupMap groups;
  for (Request* r : S->running)
    if (r->P->stream == sm)
      groups[std::make_tuple(r->n[0], r->n[1], r->n[2], r->iso, r->job.P->h16)].push_back(&r->job);
  if (groups.empty()) return FFTH_OK;
  Stage& stage = S->stages[k];
  stage.cursor = 0;
  std::vector<int> kin(groups.size(), 0);
  std::vector<InnerSet> inner(groups.size());
  const bool merge = S->opts.scheme == FFTH_CG;
  std::map<std::tuple<bool, bool>, int> sharing;
  std::vector<bool> eligible(groups.size(), false);
  size_t gi = 0;
  for (auto& kv : groups) {
    const ffth_plan* P0 = kv.second[0]->P;
    bool in = false;
    for (const Job* J : kv.second) in = in || J->phase == PH_INNER;
    eligible[gi] = merge && in && multi_grid(P0->n);
    if (eligible[gi]) ++sharing[std::make_tuple(P0->iso, P0->h16)];
    ++gi;
  }
  ffth_status st;
  gi = 0;
  for (auto& kv : groups) {
    const ffth_plan* P0 = kv.second[0]->P;
    const bool defer = eligible[gi] && sharing[std::make_tuple(P0->iso, P0->h16)] >= 2;
    if ((st = group_issue(kv.second, stage, &kin[gi], defer ? &inner[gi] : nullptr)) != FFTH_OK) return st;
    ++gi;
  }
  if (merge && (st = issue_merged(S, stage, groups, inner, kin)) != FFTH_OK) return st;
  HIPCHK(hipEventRecord(R.done, sm));
  R.busy = true;
  R.groups.clear();
  for (auto& kv : groups) R.groups.push_back(kv.second);
  R.kin = kin;
  return FFTH_OK;
}

// Complete stream k's round once its event has passed: phase transitions of
// its groups (their states were read back by the round), then the finished
// requests on the stream (volume averages, results, memory back to the arena).
ffth_status complete_round(ffth_server* S, size_t k) {
  ffth_server::Round& R = S->rounds[k];
  if (!R.busy) return FFTH_OK;
  R.busy = false;
  ffth_status st;
  for (size_t g = 0; g < R.groups.size(); ++g)
    if ((st = group_advance(R.groups[g], R.kin[g])) != FFTH_OK) return st;
  R.groups.clear();
  R.kin.clear();
  std::vector<Request*> still;
  for (Request* r : S->running) {
    if (r->P->stream != S->streams[k] || r->job.phase != PH_DONE) {
      still.push_back(r);
      continue;
    }
    r->res.assign(r->nl, ffth_result{});
    ffth_status fs = solve_finish(r->P, r->nl, r->eps, r->res.data(), r->t_submit, nullptr);
    finish_request(S, r, fs);
  }
  S->running.swap(still);
  return FFTH_OK;
}

size_t stream_index(const ffth_server* S, hipStream_t sm) {
  for (size_t k = 0; k < S->streams.size(); ++k)
    if (S->streams[k] == sm) return k;
  return 0;
}

}  // namespace

extern "C" {

size_t ffth_request_bytes(const int32_t n[3], int32_t nphases, int32_t nloads, const ffth_opts* o) {
  if (!n || !o || nloads < 1 || nphases < 1 || nphases > 65535) return 0;
  int nn[3] = {n[0], n[1], n[2]};
  if (!grid_supported(nn) || !opts_valid(*o)) return 0;
  return request_bytes(nn, nphases, nloads, *o, nullptr);
}

ffth_status ffth_server_create(ffth_server** out, void* arena, size_t arena_bytes, const ffth_opts* o,
                               int32_t max_running, void* hip_stream) {
  g_last_error.clear();
  if (!out || !arena || !o || max_running < 1) {
    g_last_error = "bad argument";
    return FFTH_ERR_INVALID;
  }
  *out = nullptr;
  if (((uintptr_t)arena) % ALIGN || !opts_valid(*o) || o->precision != FFTH_MIXED) {
    g_last_error = "arena must be 256-byte aligned; serving runs the mixed-precision solver";
    return FFTH_ERR_INVALID;
  }
  // every running request has at most 6 loads, each staged at most twice per
  // round; any one stream may carry all of them, and the rounds of different
  // streams are in flight together, so each stream has a staging area of its own
  const int cap = 12 * max_running;
  const size_t one = al((size_t)cap * sizeof(Desc));
  const size_t stage_bytes = one * FFTH_SERVER_STREAMS;
  if (arena_bytes <= stage_bytes) {
    g_last_error = "arena too small";
    return FFTH_ERR_OOM;
  }
  ffth_server* S = new ffth_server();
  S->arena = (char*)arena;
  S->bytes = arena_bytes;
  S->stream = (hipStream_t)hip_stream;
  S->opts = *o;
  S->max_running = max_running;
  S->max_bypass = max_running;
  S->stage_bytes = stage_bytes;
  S->rounds.resize(FFTH_SERVER_STREAMS);
  S->stages.assign(FFTH_SERVER_STREAMS, Stage{nullptr, nullptr, cap, 0});
  bool ok = true;
  for (int i = 0; i < FFTH_SERVER_STREAMS && ok; ++i) {
    S->stages[i].d = (Desc*)(S->arena + (size_t)i * one);
    ok = hip_ok(hipHostMalloc((void**)&S->stages[i].h, (size_t)cap * sizeof(Desc), hipHostMallocDefault),
                "hipHostMalloc") &&
         hip_ok(hipEventCreateWithFlags(&S->rounds[i].done, hipEventDisableTiming), "hipEventCreate");
  }
  S->streams.push_back(S->stream);
  for (int i = 1; i < FFTH_SERVER_STREAMS && ok; ++i) {
    hipStream_t st;
    // default priority, no implicit synchronisation with the null stream
    ok = hip_ok(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    if (ok) S->streams.push_back(st);
  }
  ok = ok && hip_ok(hipStreamCreateWithFlags(&S->admit_stream, hipStreamNonBlocking), "hipStreamCreate");
  if (!ok) {
    if (S->admit_stream) (void)hipStreamDestroy(S->admit_stream);
    for (size_t j = 1; j < S->streams.size(); ++j) (void)hipStreamDestroy(S->streams[j]);
    for (auto& st : S->stages)
      if (st.h) (void)hipHostFree(st.h);
    for (auto& r : S->rounds)
      if (r.done) (void)hipEventDestroy(r.done);
    delete S;
    return FFTH_ERR_DEVICE;
  }
  S->free_.reset(stage_bytes, arena_bytes - stage_bytes);
  *out = S;
  return FFTH_OK;
}

ffth_status ffth_submit(ffth_server* S, const ffth_problem* p, int32_t nloads, const double* E, uint64_t* id) {
  g_last_error.clear();
  if (!S || !p || !E || !id || nloads < 1 || nloads > 6) {
    g_last_error = "bad argument (1..6 load cases per request)";
    return FFTH_ERR_INVALID;
  }
  {
    int nn[3] = {p->n[0], p->n[1], p->n[2]};
    if (!grid_supported(nn)) {
      g_last_error = "unsupported grid size";
      return FFTH_ERR_INVALID;
    }
  }
  if (p->nphases < 1 || p->nphases > 65535 || !p->phase || ((p->lame == nullptr) == (p->stiffness == nullptr))) {
    g_last_error = "bad phase table";
    return FFTH_ERR_INVALID;
  }
  Request* r = new Request();
  r->id = S->next++;
  r->nl = nloads;
  for (int d = 0; d < 3; ++d) r->n[d] = p->n[d];
  r->iso = p->lame != nullptr;
  r->prob = *p;
  const int per = r->iso ? 2 : 21;
  r->table.assign(r->iso ? p->lame : p->stiffness, (r->iso ? p->lame : p->stiffness) + (size_t)per * p->nphases);
  r->E.assign(E, E + 6 * nloads);
  r->bytes = request_bytes(r->n, p->nphases, nloads, S->opts, &r->ws_bytes);
  r->t_submit = now_s();
  if (r->bytes > S->bytes - S->stage_bytes) {
    delete r;
    g_last_error = "request larger than the whole arena";
    return FFTH_ERR_OOM;
  }
  S->reqs[r->id] = r;
  S->waiting.push_back(r);
  *id = r->id;
  return FFTH_OK;
}

ffth_status ffth_server_step(ffth_server* S, int32_t* running, int32_t* waiting) {
  g_last_error.clear();
  if (!S) return FFTH_ERR_INVALID;
  ffth_status st = admit(S);
  if (st != FFTH_OK) return st;
  // idle streams with running requests start a round
  for (size_t k = 0; k < S->streams.size(); ++k)
    if (!S->rounds[k].busy && (st = issue_round(S, k)) != FFTH_OK) return st;
  // every round that has finished is completed and its stream goes on; if
  // none has, the events are polled until one has, so that whichever stream
  // finishes first is the first to go on
  for (bool done_any = false; !done_any;) {
    bool busy = false;
    for (size_t k = 0; k < S->streams.size(); ++k) {
      if (!S->rounds[k].busy) continue;
      busy = true;
      const hipError_t q = hipEventQuery(S->rounds[k].done);
      if (q == hipErrorNotReady) continue;
      HIPCHK(q);
      if ((st = complete_round(S, k)) != FFTH_OK || (st = admit(S)) != FFTH_OK || (st = issue_round(S, k)) != FFTH_OK)
        return st;
      done_any = true;
    }
    if (!busy) break;
    if (!done_any) std::this_thread::yield();
  }
  if (running) *running = (int32_t)S->running.size();
  if (waiting) *waiting = (int32_t)S->waiting.size();
  return FFTH_OK;
}

ffth_status ffth_server_stats(ffth_server* S, int64_t* multi_iterations, int32_t* multi_max_grids) {
  if (!S || !multi_iterations || !multi_max_grids) return FFTH_ERR_INVALID;
  *multi_iterations = S->multi_iterations;
  *multi_max_grids = S->multi_max_grids;
  return FFTH_OK;
}

ffth_status ffth_poll(ffth_server* S, uint64_t id, ffth_result* res) {
  if (!S) return FFTH_ERR_INVALID;
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return FFTH_ERR_INVALID;
  Request* r = it->second;
  if (r->state < 2) return FFTH_ERR_BUSY;
  ffth_status st = r->status;
  if (r->state == 2 && res)
    for (int l = 0; l < r->nl; ++l) res[l] = r->res[l];
  S->reqs.erase(it);
  delete r;
  return st;
}

ffth_status ffth_cancel(ffth_server* S, uint64_t id) {
  if (!S) return FFTH_ERR_INVALID;
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return FFTH_ERR_INVALID;
  Request* r = it->second;
  if (r->state == 1) {
    // a running request may be in its stream's round: that round completes first
    const size_t k = stream_index(S, r->P->stream);
    if (S->rounds[k].busy) {
      HIPCHK(hipEventSynchronize(S->rounds[k].done));
      ffth_status st = complete_round(S, k);
      if (st != FFTH_OK) return st;
    }
  }
  if (r->state >= 2) return FFTH_OK;
  if (r->state == 0) {
    S->waiting.erase(std::find(S->waiting.begin(), S->waiting.end(), r));
  } else {
    S->running.erase(std::find(S->running.begin(), S->running.end(), r));
  }
  finish_request(S, r, FFTH_ERR_CANCELLED);
  return FFTH_OK;
}

ffth_status ffth_server_destroy(ffth_server* S) {
  if (!S) return FFTH_ERR_INVALID;
  for (hipStream_t sm : S->streams) (void)hipStreamSynchronize(sm);   // rounds still in flight
  for (auto& kv : S->reqs) {
    Request* r = kv.second;
    if (r->P) (void)ffth_plan_destroy(r->P);
    delete r;
  }
  S->hpool.release();
  (void)hipStreamDestroy(S->admit_stream);
  for (size_t j = 1; j < S->streams.size(); ++j) (void)hipStreamDestroy(S->streams[j]);
  for (auto& st : S->stages) (void)hipHostFree(st.h);
  for (auto& rd : S->rounds) (void)hipEventDestroy(rd.done);
  delete S;
  return FFTH_OK;
}

}  // extern "C"
