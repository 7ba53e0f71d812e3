// Launch interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmc_device.h"

namespace pmc {

// Arguments of the Monte Carlo kernels, type-erased (reals are float or
// double according to the precision the launcher is called with).
struct McLaunch {
  const Instr* code;
  const void* consts;         // real[n_consts]
  const InstDesc* desc;       // per instance
  const int32_t* itab;        // packed int tables
  const void* rtab;           // packed real tables
  const double* chol;         // packed FP64 Cholesky factors
  const double* chol_in;      // packed FP64 correlation matrices (factored on device)
  int* status;                // per instance: positive-definiteness status (factor = 1)
  int factor;                 // 1: the MC kernel factors instance 0's matrix per block (no prep)
  const uint32_t* sobol;      // direction numbers [dim][32]
  int sobol_bits;             // bits of the largest path index
  const uint32_t* sobol_hi;   // per-wave high-part table [path/64][dim], or nullptr
  int sobol_dims;             // row length of sobol_hi
  const int* order;           // instance order (item i -> order[i / tiles], tile i % tiles),
                              // or nullptr: item = (instance 0, tile = block)
  int tiles;                  // tiles per instance
  int n_work;
  uint32_t* queue;            // work counter (persistent launch) or nullptr
  double2* partial;           // per item: (sum, sum of squares)
  uint32_t* done;             // batches: per-instance finished-tile counter (zeroed by launch_prep)
  double2* result;            // per instance: (sum, sum of squares); may be mapped host memory
  void* payoff_out;           // optional per-path payoffs of instance 0
  const void* paths;          // stored prices [slot][asset][path] (two-phase)
  uint32_t k0, k1;            // Philox key
  int ppt;                    // paths per thread per item
  int n_assets;
  int n_regs;                 // registers the program uses (selects the file size)
};

// A resolved Monte Carlo launch: a run-time compiled kernel (jit) or the
// static interpreter kernel of (prec, rng, mem), and the grid.
struct EngineLaunch {
  hipFunction_t f = nullptr;
  bool jit = false, mem = false;
  int prec = 0, rng = 0, grid = 0, block = 0;
};

hipError_t launch_mc(int precision, int rng, bool from_memory, const McLaunch& a, int grid, int block,
                     hipStream_t s);
// Launch of a run-time compiled Monte Carlo kernel (generated payoff).
hipError_t launch_mc_jit(hipFunction_t f, int precision, const McLaunch& a, int grid, int block, hipStream_t s);
hipError_t launch_pathgen(int precision, int rng, const McLaunch& a, void* paths, uint32_t* words,
                          void* normals, uint32_t n_paths, int block, hipStream_t s);
// Zeroes zero[0..n_zero) and factors the n correlation matrices a (m x m,
// FP64) into l; status[i] = 0 if matrix i is positive definite, else 1.
hipError_t launch_prep(const double* a, double* l, int* status, uint32_t* zero, int n_zero, int n, int m,
                       hipStream_t s);
// Sums partial[0..n) (per-block (sum, sum of squares) of a single-instrument
// launch) in order into result[0].
hipError_t launch_finish(const double2* partial, int n, double2* result, hipStream_t s);
// hi[h][d] = XOR of sobol[d][b] over the set bits b >= 6 of gray(64 h).
hipError_t launch_sobol_hi(const uint32_t* sobol, uint32_t* hi, int n_rows, int dims, int bits, hipStream_t s);
// Largest resident blocks per CU for the persistent MC kernel.
int mc_occupancy(int precision, int rng, int n_assets, int n_regs, int block);
int mc_occupancy_jit(hipFunction_t f, int block);

// Device scratch of the allocation-free pricing call: one array per device,
// of kScratchBytes, held until the process ends.  Layout: the result
// (sum, sum of squares) and the factorisation status in the first
// kScratchHead bytes, then kScratchPartials per-block partials, then the
// call's tables (bytecode, descriptors, time and discount tables,
// correlation, Sobol direction numbers) in the rest.
constexpr size_t kScratchHead = 256;
constexpr int kScratchPartials = 1 << 16;
constexpr size_t kScratchTables = size_t(2) << 20;
constexpr size_t kScratchBytes = kScratchHead + size_t(kScratchPartials) * 16 + kScratchTables;
// The device address of the scratch on `device`, which must be the current
// device.  Looked up once per device (later calls return the kept address).
hipError_t scratch_address(int device, void** out);

}  // namespace pmc
