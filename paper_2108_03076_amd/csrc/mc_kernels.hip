// Monte Carlo valuation kernels for gfx950 (MI355X, wave64).
//
// One lane evaluates one path.  The payoff expression runs as bytecode on a
// wavefront-uniform program counter: every lane of a wave executes the same
// instruction (fetched with scalar loads), conditionals are predicated with
// ballot-based skips, and a loopif iterates on a uniform shift t0 with a
// per-lane "done" mask, leaving the loop when every lane is done (the
// semantics of Fig. 3; the while-loop form of the Futhark backend, Sec. 6.2).
// Path values reach the interpreter through a per-lane window of kWindow
// registers that is refilled either by generating the path (Philox or Sobol
// words -> uniforms -> AS241 normals -> Cholesky correlation -> log-Euler
// GBM steps) or by loading stored prices [slot][asset][path].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "kernels.h"
#include "mc_engine.h"

namespace pmc {
namespace {
using namespace eng;

template <typename T>
Args<T> typed(const McLaunch& a) {
  Args<T> g;
  g.code = a.code; g.consts = (const T*)a.consts; g.desc = a.desc; g.itab = a.itab;
  g.rtab = (const T*)a.rtab; g.chol = a.chol; g.sobol = a.sobol; g.sobol_bits = a.sobol_bits;
  g.order = a.order; g.tiles = a.tiles; g.n_work = a.n_work; g.queue = a.queue; g.partial = a.partial;
  g.done = a.done; g.result = a.result;
  g.chol_in = a.chol_in; g.status = a.status; g.factor = a.factor;
  g.payoff_out = (T*)a.payoff_out; g.paths = (const T*)a.paths; g.k0 = a.k0; g.k1 = a.k1;
  g.ppt = a.ppt; g.n_assets = a.n_assets;
  g.sobol_hi = a.sobol_hi; g.sobol_dims = a.sobol_dims;
  return g;
}

template <typename T, int RNG, int A, bool MEM, int NR>
__global__ __launch_bounds__(256) void k_mc(Args<T> g) {
  mc_body<T, RNG, A, MEM, Interp<NR>>(g);
}

template <typename T, int RNG, int A>
__global__ __launch_bounds__(256) void k_pathgen(Args<T> g, T* out, uint32_t* wout, T* zout, uint32_t n_paths) {
  pathgen_body<T, RNG, A>(g, out, wout, zout, n_paths);
}

// Prepares a launch: zeroes n_zero work counters and factors every
// instance's correlation matrix (FP64 Cholesky-Banachiewicz, one matrix per
// thread).  status[i] = 0 if matrix i is positive definite, else 1.  A kernel
// rather than a memset, so that the sequence can be captured into a graph.
__global__ void k_prep(const double* a, double* l, int* status, uint32_t* zero, int n_zero, int n, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_zero) zero[i] = 0u;
  if (i >= n) return;
  const bool ok = chol_factor(a + (size_t)i * m * m, l + (size_t)i * m * m, m);
  status[i] = ok ? 0 : 1;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");   // system scope: host-mapped memory
}

// Sums the n per-block partials of a single-instrument launch in block order
// (a fixed order: deterministic) and writes the instrument's result, which
// may be host-mapped memory; the host reads it after waiting on an event
// recorded behind this kernel, whose system-scope release publishes it (no
// fence here: an in-kernel one writes back the whole L2).  One block of
// kFinishThreads.
constexpr int kFinishThreads = 256;
__global__ __launch_bounds__(kFinishThreads) void k_finish(const double2* partial, int n, double2* result) {
  __shared__ double red[8];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double2 q = partial[i];
    a += q.x; b += q.y;
  }
  block_sum2(a, b, red);
  if (threadIdx.x == 0) result[0] = make_double2(a, b);
}

__global__ void k_sobol_hi(const uint32_t* v, uint32_t* hi, int n_rows, int dims, int bits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows * dims) return;
  const uint32_t h = (uint32_t)(i / dims), d = (uint32_t)(i % dims);
  const uint32_t gh = h ^ (h >> 1);   // Gray-code bits 6.. of points 64h .. 64h+63
  uint32_t acc = 0;
  for (int b = 6; b < bits; ++b)
    if ((gh >> (b - 6)) & 1u) acc ^= v[d * 32u + b];
  hi[i] = acc;
}

template <typename T, int RNG, int A>
hipError_t mc_launch_t(bool mem, const McLaunch& a, int grid, int block, hipStream_t s) {
  Args<T> g = typed<T>(a);
  const bool small = a.n_regs <= 7;   // user registers 0..6, sink 31 -> 7
  if (mem) {
    if (small) hipLaunchKernelGGL((k_mc<T, RNG, A, true, 8>), dim3(grid), dim3(block), 0, s, g);
    else hipLaunchKernelGGL((k_mc<T, RNG, A, true, 32>), dim3(grid), dim3(block), 0, s, g);
  } else {
    if (small) hipLaunchKernelGGL((k_mc<T, RNG, A, false, 8>), dim3(grid), dim3(block), 0, s, g);
    else hipLaunchKernelGGL((k_mc<T, RNG, A, false, 32>), dim3(grid), dim3(block), 0, s, g);
  }
  return hipGetLastError();
}

template <typename T, int RNG>
hipError_t mc_launch_a(bool mem, const McLaunch& a, int grid, int block, hipStream_t s) {
  switch (a.n_assets) {
    case 1: return mc_launch_t<T, RNG, 1>(mem, a, grid, block, s);
    case 2: return mc_launch_t<T, RNG, 2>(mem, a, grid, block, s);
    case 3: return mc_launch_t<T, RNG, 3>(mem, a, grid, block, s);
    case 4: return mc_launch_t<T, RNG, 4>(mem, a, grid, block, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int RNG, int A>
hipError_t pg_launch_t(const McLaunch& a, void* paths, uint32_t* words, void* normals, uint32_t n,
                       int block, hipStream_t s) {
  Args<T> g = typed<T>(a);
  const int grid = (int)((n + block - 1) / block);
  hipLaunchKernelGGL((k_pathgen<T, RNG, A>), dim3(grid), dim3(block), 0, s, g, (T*)paths, words,
                     (T*)normals, n);
  return hipGetLastError();
}

template <typename T, int RNG>
hipError_t pg_launch_a(const McLaunch& a, void* paths, uint32_t* words, void* normals, uint32_t n,
                       int block, hipStream_t s) {
  switch (a.n_assets) {
    case 1: return pg_launch_t<T, RNG, 1>(a, paths, words, normals, n, block, s);
    case 2: return pg_launch_t<T, RNG, 2>(a, paths, words, normals, n, block, s);
    case 3: return pg_launch_t<T, RNG, 3>(a, paths, words, normals, n, block, s);
    case 4: return pg_launch_t<T, RNG, 4>(a, paths, words, normals, n, block, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int RNG, int A>
int occ_t(int block, int n_regs) {
  int n = 0;
  hipError_t e = n_regs <= 7
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mc<T, RNG, A, false, 8>, block, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mc<T, RNG, A, false, 32>, block, 0);
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

// The allocation-free call's scratch.  In host code `scratch` names a
// host-side stand-in, not device memory: only the address that
// hipGetSymbolAddress returns for the current device is ever passed to a
// kernel or a copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

}  // namespace

hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;   // per device
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p || ((uintptr_t)p & 255u)) return hipErrorInvalidSymbol;
  addr[device] = p;
  *out = p;
  return hipSuccess;
}

hipError_t launch_mc(int precision, int rng, bool mem, const McLaunch& a, int grid, int block,
                     hipStream_t s) {
  if (block % 64 != 0 || block > 256 || block <= 0) return hipErrorInvalidValue;
  if (precision == 1) return rng ? mc_launch_a<double, 1>(mem, a, grid, block, s) : mc_launch_a<double, 0>(mem, a, grid, block, s);
  return rng ? mc_launch_a<float, 1>(mem, a, grid, block, s) : mc_launch_a<float, 0>(mem, a, grid, block, s);
}

hipError_t launch_pathgen(int precision, int rng, const McLaunch& a, void* paths, uint32_t* words,
                          void* normals, uint32_t n, int block, hipStream_t s) {
  if (precision == 1) return rng ? pg_launch_a<double, 1>(a, paths, words, normals, n, block, s) : pg_launch_a<double, 0>(a, paths, words, normals, n, block, s);
  return rng ? pg_launch_a<float, 1>(a, paths, words, normals, n, block, s) : pg_launch_a<float, 0>(a, paths, words, normals, n, block, s);
}

hipError_t launch_mc_jit(hipFunction_t f, int precision, const McLaunch& a, int grid, int block, hipStream_t s) {
  if (block % 64 != 0 || block > 256 || block <= 0) return hipErrorInvalidValue;
  if (precision == 1) {
    Args<double> g = typed<double>(a);
    void* params[] = {&g};
    return hipModuleLaunchKernel(f, grid, 1, 1, block, 1, 1, 0, s, params, nullptr);
  }
  Args<float> g = typed<float>(a);
  void* params[] = {&g};
  return hipModuleLaunchKernel(f, grid, 1, 1, block, 1, 1, 0, s, params, nullptr);
}

hipError_t launch_prep(const double* a, double* l, int* status, uint32_t* zero, int n_zero, int n, int m,
                       hipStream_t s) {
  const int t = std::max(n, n_zero);
  hipLaunchKernelGGL(k_prep, dim3((t + 255) / 256), dim3(256), 0, s, a, l, status, zero, n_zero, n, m);
  return hipGetLastError();
}

hipError_t launch_finish(const double2* partial, int n, double2* result, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishThreads), 0, s, partial, n, result);
  return hipGetLastError();
}

hipError_t launch_sobol_hi(const uint32_t* sobol, uint32_t* hi, int n_rows, int dims, int bits, hipStream_t s) {
  const int n = n_rows * dims;
  hipLaunchKernelGGL(k_sobol_hi, dim3((n + 255) / 256), dim3(256), 0, s, sobol, hi, n_rows, dims, bits);
  return hipGetLastError();
}

int mc_occupancy(int precision, int rng, int n_assets, int n_regs, int block) {
#define OCC(T, R) \
  switch (n_assets) { case 1: return occ_t<T, R, 1>(block, n_regs); case 2: return occ_t<T, R, 2>(block, n_regs); \
                      case 3: return occ_t<T, R, 3>(block, n_regs); default: return occ_t<T, R, 4>(block, n_regs); }
  if (precision == 1) { if (rng) { OCC(double, 1) } else { OCC(double, 0) } }
  if (rng) { OCC(float, 1) } else { OCC(float, 0) }
#undef OCC
}

int mc_occupancy_jit(hipFunction_t f, int block) {
  int n = 0;
  if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace pmc