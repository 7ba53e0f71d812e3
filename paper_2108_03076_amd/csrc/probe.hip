// Peak-rate probes: the vector-ALU issue rate this GPU sustains for the
// instruction classes the Monte Carlo kernels are made of, measured by
// kernels of independent dependency chains on every SIMD (no memory traffic
// in the timed loop), and the device-to-device copy bandwidth.  They back
// the roofline figures the benchmark reports beside the published peaks.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/pmc.h"
#include "ctx.h"

namespace {

constexpr int kChains = 8;
constexpr int kProbeBlocks = 2048;   // 8 per CU on 256 CUs
constexpr int kProbeThreads = 256;

// kind 0: v_fma_f32; 1: v_xor_b32 (+ v_add_u32 to keep the chains live);
// 2: v_mad_u64_u32 (32 x 32 -> 64 products); 3: v_exp_f32; 4: v_fma_f32 and
// v_xor_b32 chains interleaved
__global__ __launch_bounds__(kProbeThreads) void k_probe(int kind, int iters, float* sink) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  float f[kChains];
  uint32_t u[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    f[c] = (float)(t & 255u) * 1e-3f + (float)c;
    u[c] = t * 2654435761u + (uint32_t)c;
  }
  const float fa = sink[0], fb = sink[1];
  const uint32_t ua = __float_as_uint(sink[2]) | 1u, ub = __float_as_uint(sink[3]);
  if (kind == 0) {
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) f[c] = fmaf(f[c], fa, fb);
    }
  } else if (kind == 1) {
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) u[c] = (u[c] ^ ua) + ub;
    }
  } else if (kind == 2) {
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        const uint64_t p = (uint64_t)u[c] * ua + ub;   // one v_mad_u64_u32
        u[c] = (uint32_t)(p >> 32) + (uint32_t)p;
      }
    }
  } else if (kind == 3) {
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) f[c] = __builtin_amdgcn_exp2f(f[c]) * fa;
    }
  } else {
    // FMA and integer chains interleaved (independent instruction types)
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        f[c] = fmaf(f[c], fa, fb);
        u[c] = u[c] ^ ua;
      }
    }
  }
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc += f[c] + (float)(u[c] & 1u);
  if (acc == 123.456f) sink[4] = acc;   // never true; keeps the chains live
}

}  // namespace

extern "C" int pmc_probe_valu(pmc_ctx* c, int kind, double* lane_ops_per_s) {
  if (!c || !lane_ops_per_s || kind < 0 || kind > 4) return PMC_E_ARG;
  hipStream_t s = pmc::ctx_stream(c);
  auto hip = [&](hipError_t e) {
    return e == hipSuccess ? PMC_OK : pmc::ctx_fail(c, PMC_E_HIP, std::string("probe: ") + hipGetErrorString(e));
  };
  int st = hip(hipSetDevice(pmc::ctx_device(c)));
  if (st != PMC_OK) return st;
  float* sink = nullptr;
  if ((st = hip(hipMalloc(&sink, 8 * sizeof(float)))) != PMC_OK) return st;
  const float init[8] = {0.999f, 1e-3f, 1.7f, 3.1f, 0, 0, 0, 0};
  hipEvent_t a = nullptr, b = nullptr;
  const int iters = kind == 3 ? 1 << 12 : 1 << 14;
  float ms = 0;
  st = hip(hipMemcpyAsync(sink, init, sizeof init, hipMemcpyHostToDevice, s));
  if (st == PMC_OK) st = hip(hipEventCreate(&a));
  if (st == PMC_OK) st = hip(hipEventCreate(&b));
  if (st == PMC_OK) {
    hipLaunchKernelGGL(k_probe, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, kind, 16, sink);   // warm-up
    st = hip(hipEventRecord(a, s));
  }
  if (st == PMC_OK) {
    hipLaunchKernelGGL(k_probe, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, kind, iters, sink);
    st = hip(hipGetLastError());
  }
  if (st == PMC_OK) st = hip(hipEventRecord(b, s));
  if (st == PMC_OK) st = hip(hipEventSynchronize(b));
  if (st == PMC_OK) st = hip(hipEventElapsedTime(&ms, a, b));
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(sink);
  if (st != PMC_OK) return st;
  // lane operations of the timed loop: per chain and iteration one FMA
  // (kind 0) or two instructions (kind 1: xor, add; 2: product, add; 3:
  // exp2, multiply; 4: FMA, xor)
  const double per = kind == 0 ? 1.0 : 2.0;
  *lane_ops_per_s = per * (double)kChains * iters * (double)kProbeBlocks * kProbeThreads / (ms * 1e-3);
  return PMC_OK;
}
