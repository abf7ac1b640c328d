// ffth_green_apply_noalloc: the Green operator application of
// ffth_green_apply without a plan or a caller workspace, for callers that
// cannot allocate device memory.  Everything the passes need beyond the input
// and output fields (launch descriptor, gating state, block partial sums, a
// zero phase array and the half spectrum) lives in one file-scope device
// array of fixed size, one copy per GPU, held until the process ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "ffth.h"
#include "ffth_launch.h"
#include "ffth_types.h"

using namespace ffth;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t al(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Regions of the scratch array for the largest grid: descriptor, state,
// forward and inverse partial sums (NRED doubles per x-pass block; blocks <=
// rows = n0 n1 <= voxels / 4), the phase ids (zero: the copy-in pass reads
// them) and the FP64 half spectrum (48 bytes per voxel).
constexpr size_t kVox = FFTH_NOALLOC_MAX_VOXELS;
constexpr size_t kRows = kVox / 4;
constexpr size_t kOffDesc = 0;
constexpr size_t kOffState = al(sizeof(Desc));
constexpr size_t kOffPartF = kOffState + al(sizeof(SolverState));
constexpr size_t kOffPartI = kOffPartF + al(kRows * NRED * sizeof(double));
constexpr size_t kOffPhase = kOffPartI + al(kRows * NRED * sizeof(double));
constexpr size_t kOffSpec = kOffPhase + al(kVox * sizeof(uint16_t));
constexpr size_t kBytes = kOffSpec + al(kVox * 6 * sizeof(double));

static_assert(kBytes == FFTH_NOALLOC_SCRATCH_BYTES, "scratch size stated in ffth.h");

static __device__ __align__(256) unsigned char scratch[kBytes];

// Device address of `scratch` per GPU (its name is a host-side stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

// Descriptor and state go to scratch from the kernel arguments (no host
// buffer has to outlive the call); the phase ids of the grid are cleared.
__global__ void k_noalloc_setup(Desc d, SolverState s, Desc* dd, SolverState* ss, uint16_t* phase, long nvox) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *dd = d;
    *ss = s;
  }
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nvox; i += (long)gridDim.x * blockDim.x)
    phase[i] = 0;
}

int kchunk_of(int h) {
  int c = h < 16 ? h : 16;
  while (h % c) --c;
  return c;
}

template <typename T> hipError_t green_passes(const int n[3], hipStream_t st, const Desc* d) {
  const long rows = (long)n[0] * n[1], nvox = rows * n[2];
  const int h = n[2] / 2, kc = kchunk_of(h);
  const int xr = Launch<T>::x_rows(n[2], 0), xir = Launch<T>::xi_rows(n[2], 0);
  hipError_t e;
  if ((e = Launch<T>::xfwd(n[2], true, 0, false, dim3((unsigned)((rows + xr - 1) / xr), 1), st, d, XF_COPY, rows,
                           nvox)) != hipSuccess)
    return e;
  const int ncols = kc * 6, nplanes = n[0] * (h / kc);
  const int cw = Launch<T>::y_cols(n[1], 0), ntiles = (ncols + cw - 1) / cw;
  if ((e = Launch<T>::ypass(n[1], 0, false, dim3(nplanes * ntiles, 1), st, d, -1, ncols, ntiles)) != hipSuccess)
    return e;
  const long M = (long)n[1] * kc;
  const int tk = Launch<T>::z_cols(n[0], 0);
  const int nzb = (int)((M + tk - 1) / tk) * (h / kc);
  if ((e = Launch<T>::zpass(n[0], 0, false, dim3(nzb, 1), st, d, OP_GAMMA, n[1], h, 1.0 / (double)nvox)) !=
      hipSuccess)
    return e;
  if ((e = Launch<T>::ypass(n[1], 0, false, dim3(nplanes * ntiles, 1), st, d, +1, ncols, ntiles)) != hipSuccess)
    return e;
  return Launch<T>::xinv(n[2], true, 0, dim3((unsigned)((rows + xir - 1) / xir), 1), st, d, XI_STORE, rows, nvox);
}

ffth_status fail(ffth_status s, const std::string& msg) {
  set_last_error(msg.c_str());
  return s;
}

}  // namespace

extern "C" {

ffth_status ffth_green_apply_noalloc(const int32_t n[3], double lambda0, double mu0, const double* tau, double* eta,
                                     int32_t precision, void* hip_stream) {
  set_last_error("");
  if (!n || !tau || !eta) return fail(FFTH_ERR_INVALID, "null argument");
  if (precision != FFTH_FP64 && precision != FFTH_FP32) return fail(FFTH_ERR_INVALID, "precision must be FP64 or FP32");
  int nn[3] = {n[0], n[1], n[2]};
  if (!grid_supported(nn)) return fail(FFTH_ERR_INVALID, "unsupported grid");
  const long nvox = (long)nn[0] * nn[1] * nn[2];
  if (nvox > (long)FFTH_NOALLOC_MAX_VOXELS)
    return fail(FFTH_ERR_INVALID, "grid of " + std::to_string(nvox) + " voxels exceeds the " +
                                      std::to_string((long)FFTH_NOALLOC_MAX_VOXELS) +
                                      "-voxel limit of the allocation-free entry point");
  if (!(mu0 != 0.0) || !(lambda0 + 2.0 * mu0 != 0.0) || !std::isfinite(mu0) || !std::isfinite(lambda0))
    return fail(FFTH_ERR_INVALID, "reference medium needs mu0 != 0 and lambda0 + 2 mu0 != 0");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(FFTH_ERR_DEVICE, "no usable device");
  char* base;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return fail(FFTH_ERR_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
      g_ptr[dev] = p;
    }
    base = (char*)g_ptr[dev];
  }
  hipStream_t st = (hipStream_t)hip_stream;
  Desc d;
  std::memset(&d, 0, sizeof(d));
  d.phase = (const uint16_t*)(base + kOffPhase);
  d.spec = base + kOffSpec;
  d.part_f = (double*)(base + kOffPartF);
  d.part_i = (double*)(base + kOffPartI);
  d.st = (SolverState*)(base + kOffState);
  d.io = (void*)tau;
  d.out = eta;
  d.nc = 6;
  d.lam0 = lambda0;
  d.mu0 = mu0;
  d.inv_nvox = 1.0 / (double)nvox;
  d.tau_scale = 1.0;
  d.op_scale = 1.0 / (double)nvox;
  SolverState s;
  std::memset(&s, 0, sizeof(s));
  s.active = 1;
  s.first = 1;
  s.max_iter = 1;
  s.res = 1.0;
  s.dscale = 1.0;
  s.gscale = -1.0;
  const int nb = (int)std::min<long>(1024, (nvox + 255) / 256);
  hipLaunchKernelGGL(k_noalloc_setup, dim3(nb), dim3(256), 0, st, d, s, (Desc*)(base + kOffDesc),
                     (SolverState*)(base + kOffState), (uint16_t*)(base + kOffPhase), nvox);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = precision == FFTH_FP64 ? green_passes<double>(nn, st, (const Desc*)(base + kOffDesc))
                               : green_passes<float>(nn, st, (const Desc*)(base + kOffDesc));
  if (e != hipSuccess) return fail(FFTH_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return FFTH_OK;
}

}  // extern "C"
