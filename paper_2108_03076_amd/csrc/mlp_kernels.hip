// Surrogate MLP kernels for gfx950: BF16 x BF16 -> FP32 GEMMs on the matrix
// cores (v_mfma_f32_32x32x16_bf16) with fused epilogues (bias + GELU,
// GELU'-scaled back-propagation, split-K weight gradients), plus the input
// scaling, loss, bias-gradient, Adam and weight-packing kernels.
#include <hip/hip_runtime.h>

#include "mlp_kernels.h"

namespace pmc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }

// erf by Abramowitz & Stegun 7.1.26 (Hastings' rational form):
// erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^{-x^2},
// t = 1 / (1 + p x), x >= 0, |error| <= 1.5e-7 (far below the BF16 rounding
// of the activations it feeds); odd symmetry for x < 0.
__device__ __forceinline__ float erf_as(float v) {
  const float x = fabsf(v);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  float q = fmaf(1.061405429f, t, -1.453152027f);
  q = fmaf(q, t, 1.421413741f);
  q = fmaf(q, t, -0.284496736f);
  q = fmaf(q, t, 0.254829592f);
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * x * x);
  return copysignf(fmaf(-q * t, e, 1.0f), v);
}
// GELU with the erf form and its derivative (the same erf in training and
// inference).
__device__ __forceinline__ float gelu(float z) {
  const float h = 0.5f * z;
  return fmaf(h, erf_as(z * 0.70710678118654752f), h);
}
__device__ __forceinline__ float gelu_grad(float z) {
  return fmaf(0.5f, erf_as(z * 0.70710678118654752f), 0.5f) +
         z * 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.72134752044448170f * z * z);
}

// C = A * Bt^T with A [M x K] and Bt [N x K] row-major BF16 (K contiguous).
// Block: 4 waves on a 64 x 64 output tile, each wave one 32 x 32 MFMA tile;
// blockIdx.z splits K into chunks of k_chunk.  M, N multiples of 32, K and
// k_chunk multiples of 16, lda/ldb multiples of 8 (16-byte rows).
// MFMA operand layout (32x32x16): lane l supplies row l%32 of A (and of Bt)
// at k = 8*(l/32) .. +7; accumulator element e of lane l is
// C[8*(e/4) + 4*(l/32) + e%4][l%32].
template <class Epi>
__global__ __launch_bounds__(256) void k_gemm_nt(int M, int N, int K, const __bf16* __restrict__ A, int lda,
                                                 const __bf16* __restrict__ Bt, int ldb, int k_chunk, Epi epi) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (w & 1) * 32;
  if (m0 >= M || n0 >= N) return;
  const int kbeg = blockIdx.z * k_chunk;
  const int kend = min(K, kbeg + k_chunk);
  const int r = lane & 31, kh = (lane >> 5) * 8;
  const __bf16* pa = A + (size_t)(m0 + r) * lda + kh;
  const __bf16* pb = Bt + (size_t)(n0 + r) * ldb + kh;
  f32x16 acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
  for (int k = kbeg; k < kend; k += 16) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(pa + k);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(pb + k);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const int col = n0 + r;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = m0 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    epi(row, col, acc[e], (int)blockIdx.z);
  }
}

struct EpiF32 {          // C[z][row][col] (split-K partials or plain output)
  float* c; int ldc; size_t zstride;
  __device__ void operator()(int row, int col, float v, int z) const { c[z * zstride + (size_t)row * ldc + col] = v; }
};

struct EpiHidden {       // z = v + b; Z = z; H = gelu(z) (BF16) and its transpose
  const float* bias; float* Z; int ldz; __bf16* H; int ldh; __bf16* Ht; int ldht;
  __device__ void operator()(int row, int col, float v, int) const {
    const float z = v + bias[col];
    Z[(size_t)row * ldz + col] = z;
    const __bf16 h = to_bf16(gelu(z));
    H[(size_t)row * ldh + col] = h;
    Ht[(size_t)col * ldht + row] = h;
  }
};

struct EpiHiddenInfer {  // H = gelu(v + b) (BF16) only
  const float* bias; __bf16* H; int ldh;
  __device__ void operator()(int row, int col, float v, int) const {
    H[(size_t)row * ldh + col] = to_bf16(gelu(v + bias[col]));
  }
};

struct EpiOut {          // y = (v + b) * scale for output column 0
  const float* bias; float* y; float scale;
  __device__ void operator()(int row, int col, float v, int) const {
    if (col == 0) y[row] = (v + bias[0]) * scale;
  }
};

struct EpiBackHidden {   // dZ = dH * gelu'(Z) (BF16) and its transpose
  const float* Z; int ldz; __bf16* dZ; int lddz; __bf16* dZt; int lddzt;
  __device__ void operator()(int row, int col, float v, int) const {
    const float g = v * gelu_grad(Z[(size_t)row * ldz + col]);
    const __bf16 b = to_bf16(g);
    dZ[(size_t)row * lddz + col] = b;
    dZt[(size_t)col * lddzt + row] = b;
  }
};

template <class Epi>
hipError_t gemm(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb, int splits, Epi epi,
                hipStream_t s) {
  if (M % 32 || N % 32 || K % 16 || lda % 8 || ldb % 8 || splits < 1) return hipErrorInvalidValue;
  int chunk = (K + splits - 1) / splits;
  chunk = (chunk + 15) / 16 * 16;
  dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
  hipLaunchKernelGGL((k_gemm_nt<Epi>), grid, dim3(256), 0, s, M, N, K, A, lda, Bt, ldb, chunk, epi);
  return hipGetLastError();
}

// x raw [n][n_in] -> X [B][16] BF16 scaled to [-1,1] (columns >= n_in zero)
// and its transpose Xt [32][B] (rows >= n_in zero).  Rows >= n are zero.
__global__ void k_scale_inputs(const float* __restrict__ x, int n, int n_in, const float* __restrict__ lo,
                               const float* __restrict__ hi, int B, __bf16* X, __bf16* Xt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  for (int j = 0; j < 32; ++j) {
    float v = 0.0f;
    if (i < n && j < n_in) v = 2.0f * (x[(size_t)i * n_in + j] - lo[j]) / (hi[j] - lo[j]) - 1.0f;
    const __bf16 b = to_bf16(v);
    if (j < 16) X[(size_t)i * 16 + j] = b;
    Xt[(size_t)j * B + i] = b;
  }
}

// dy = 2 (yhat - t) / n_total for real rows (0 for padding), stored as the
// first column of dZ4 [B][32] and first row of dZ4t [32][B]; per-block sums
// of (yhat - t)^2 into part[block].
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ yhat, const float* __restrict__ t, int n,
                                              int B, float inv_scale, float grad_scale, __bf16* dZ, __bf16* dZt,
                                              double* part) {
  __shared__ double red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (i < B) {
    float d = 0.0f;
    if (i < n) {
      const float e = yhat[i] - t[i] * inv_scale;
      l = (double)e * (double)e;
      d = grad_scale * e;
    }
    const __bf16 b = to_bf16(d);
    for (int j = 0; j < 32; ++j) {
      dZ[(size_t)i * 32 + j] = j == 0 ? b : to_bf16(0.0f);
      dZt[(size_t)j * B + i] = j == 0 ? b : to_bf16(0.0f);
    }
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] += sum of part[0..n) in a fixed order (one thread).
__global__ void k_sum_parts(const double* part, int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  out[0] += s;
}

// g[row][col] (rows < rows_real, cols < cols_real, row-major ld cols_real)
// = sum over z of partial[z][row][col] (ld ldp), fixed order.
__global__ void k_reduce_splits(const float* __restrict__ partial, int splits, size_t zstride, int ldp,
                                int rows_real, int cols_real, float* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows_real * cols_real) return;
  const int row = i / cols_real, col = i % cols_real;
  float s = 0.0f;
  for (int z = 0; z < splits; ++z) s += partial[z * zstride + (size_t)row * ldp + col];
  g[i] = s;
}

// g[r] = sum over b of dZt[r][b] (BF16), one block per row, fixed order.
__global__ __launch_bounds__(256) void k_rowsum(const __bf16* __restrict__ dZt, int B, int rows_real,
                                                float* __restrict__ g) {
  __shared__ float red[256];
  const int r = blockIdx.x;
  if (r >= rows_real) return;
  float s = 0.0f;
  for (int b = threadIdx.x; b < B; b += blockDim.x) s += from_bf16(dZt[(size_t)r * B + b]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[r] = red[0];
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 working copies of a layer's weights from the FP32 master [out][in]:
// W [out_pad][in_pad] and Wt [in_pad][out_pad], zero padded.
__global__ void k_pack(const float* __restrict__ master, int out, int in, int out_pad, int in_pad, __bf16* W,
                       __bf16* Wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= out_pad * in_pad) return;
  const int o = i / in_pad, k = i % in_pad;
  const float x = (o < out && k < in) ? master[(size_t)o * in + k] : 0.0f;
  const __bf16 b = to_bf16(x);
  W[(size_t)o * in_pad + k] = b;
  Wt[(size_t)k * out_pad + o] = b;
}

// Fused inference for width 256: a block carries 128 samples through the
// four layers, their activations kept in LDS as BF16 between layers (rows
// padded by 8 elements, so the 16 rows of a half-wave's A-fragment reads
// fall on distinct banks).  Wave w computes output columns 64w .. 64w+63
// of all 128 rows: per k step it loads its two weight fragments once (each
// weight is read once per block, not once per wave) and four activation
// fragments from LDS, for eight 32 x 32 MFMA tiles.  The k order, the MFMA
// instruction and the epilogues are those of the per-layer kernels, so the
// outputs are the same bit for bit.
constexpr int kInferRows = 128;
constexpr int kInferW = 256;
constexpr int kInferLd = kInferW + 8;

// acc[rt][c]: rows 32 rt .. 32 rt + 31, columns 32 (2w + c) .. + 31; column
// tiles at or beyond ntiles (the padded output layer) are skipped.
template <int K>
__device__ __forceinline__ void infer_layer(const __bf16* act, const __bf16* __restrict__ Wl, int ntiles,
                                            f32x16 (&acc)[4][2]) {
  const int lane = threadIdx.x & 63, r = lane & 31, kh = (lane >> 5) * 8, w = threadIdx.x >> 6;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[rt][c][e] = 0.0f;
  if (2 * w >= ntiles) return;
#pragma unroll 2
  for (int k = 0; k < K; k += 16) {
    bf16x8 b[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
      if (2 * w + c < ntiles) b[c] = *reinterpret_cast<const bf16x8*>(Wl + (size_t)(32 * (2 * w + c) + r) * K + k + kh);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(act + (32 * rt + r) * kInferLd + k + kh);
#pragma unroll
      for (int c = 0; c < 2; ++c)
        if (2 * w + c < ntiles) acc[rt][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[c], acc[rt][c], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void infer_hidden_epilogue(__bf16* act, const float* __restrict__ bias,
                                                      const f32x16 (&acc)[4][2]) {
  const int lane = threadIdx.x & 63, r = lane & 31, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = 32 * (2 * w + c) + r;
    const float b = bias[col];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = 32 * rt + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        act[row * kInferLd + col] = to_bf16(gelu(acc[rt][c][e] + b));
      }
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_mlp_infer256(const float* __restrict__ x, int n, int n_in,
                                                      const float* __restrict__ lohi, const __bf16* __restrict__ W1,
                                                      const float* __restrict__ b1, const __bf16* __restrict__ W2,
                                                      const float* __restrict__ b2, const __bf16* __restrict__ W3,
                                                      const float* __restrict__ b3, const __bf16* __restrict__ W4,
                                                      const float* __restrict__ b4, float y_scale,
                                                      float* __restrict__ y) {
  __shared__ __bf16 act[kInferRows * kInferLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t g0 = (int64_t)blockIdx.x * kInferRows;   // global row of the block's first row
  {   // scaled inputs in columns 0..15 (zero beyond n_in and beyond n); wave w fills rows 32w ..
    const int row = 32 * w + (lane & 31), j0 = (lane >> 5) * 8;
    const int64_t gi = g0 + row;
#pragma unroll
    for (int j = j0; j < j0 + 8; ++j) {
      float v = 0.0f;
      if (gi < n && j < n_in) v = 2.0f * (x[gi * n_in + j] - lohi[j]) / (lohi[32 + j] - lohi[j]) - 1.0f;
      act[row * kInferLd + j] = to_bf16(v);
    }
  }
  __syncthreads();
  f32x16 acc[4][2];
  infer_layer<16>(act, W1, 8, acc);
  __syncthreads();
  infer_hidden_epilogue(act, b1, acc);
  __syncthreads();
  infer_layer<kInferW>(act, W2, 8, acc);
  __syncthreads();
  infer_hidden_epilogue(act, b2, acc);
  __syncthreads();
  infer_layer<kInferW>(act, W3, 8, acc);
  __syncthreads();
  infer_hidden_epilogue(act, b3, acc);
  __syncthreads();
  infer_layer<kInferW>(act, W4, 1, acc);   // output layer: rows of W4 padded to 32, column 0 real (wave 0)
  if (w == 0 && (lane & 31) == 0) {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = 32 * rt + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (g0 + row < n) y[g0 + row] = (acc[rt][0][e] + b4[0]) * y_scale;
      }
  }
}

}  // namespace

hipError_t mlp_gemm_f32(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb, int splits,
                        float* C, int ldc, hipStream_t s) {
  return gemm(M, N, K, A, lda, Bt, ldb, splits, EpiF32{C, ldc, (size_t)M * ldc}, s);
}
hipError_t mlp_gemm_hidden(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb,
                           const float* bias, float* Z, __bf16* H, __bf16* Ht, hipStream_t s) {
  return gemm(M, N, K, A, lda, Bt, ldb, 1, EpiHidden{bias, Z, N, H, N, Ht, M}, s);
}
hipError_t mlp_gemm_hidden_infer(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb,
                                 const float* bias, __bf16* H, hipStream_t s) {
  return gemm(M, N, K, A, lda, Bt, ldb, 1, EpiHiddenInfer{bias, H, N}, s);
}
hipError_t mlp_gemm_out(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb, const float* bias,
                        float* y, float scale, hipStream_t s) {
  return gemm(M, N, K, A, lda, Bt, ldb, 1, EpiOut{bias, y, scale}, s);
}
hipError_t mlp_gemm_back_hidden(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb,
                                const float* Z, __bf16* dZ, __bf16* dZt, hipStream_t s) {
  return gemm(M, N, K, A, lda, Bt, ldb, 1, EpiBackHidden{Z, N, dZ, N, dZt, M}, s);
}
hipError_t mlp_scale_inputs(const float* x, int n, int n_in, const float* lo, const float* hi, int B, __bf16* X,
                            __bf16* Xt, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inputs, dim3((B + 255) / 256), dim3(256), 0, s, x, n, n_in, lo, hi, B, X, Xt);
  return hipGetLastError();
}
hipError_t mlp_loss(const float* yhat, const float* t, int n, int B, float inv_scale, float grad_scale, __bf16* dZ,
                    __bf16* dZt, double* part, double* acc, hipStream_t s) {
  const int blocks = (B + 255) / 256;
  hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, s, yhat, t, n, B, inv_scale, grad_scale, dZ, dZt, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part, blocks, acc);
  return hipGetLastError();
}
hipError_t mlp_reduce_splits(const float* partial, int splits, size_t zstride, int ldp, int rows, int cols,
                             float* g, hipStream_t s) {
  const int n = rows * cols;
  hipLaunchKernelGGL(k_reduce_splits, dim3((n + 255) / 256), dim3(256), 0, s, partial, splits, zstride, ldp, rows,
                     cols, g);
  return hipGetLastError();
}
hipError_t mlp_rowsum(const __bf16* dZt, int B, int rows, float* g, hipStream_t s) {
  hipLaunchKernelGGL(k_rowsum, dim3(rows), dim3(256), 0, s, dZt, B, rows, g);
  return hipGetLastError();
}
hipError_t mlp_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t mlp_infer256(const float* x, int n, int n_in, const float* lohi, const __bf16* W1, const float* b1,
                        const __bf16* W2, const float* b2, const __bf16* W3, const float* b3, const __bf16* W4,
                        const float* b4, float y_scale, float* y, hipStream_t s) {
  if (n < 1 || n_in < 1 || n_in > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_infer256, dim3((n + kInferRows - 1) / kInferRows), dim3(256), 0, s, x, n, n_in, lohi, W1,
                     b1, W2, b2, W3, b3, W4, b4, y_scale, y);
  return hipGetLastError();
}
hipError_t mlp_pack(const float* master, int out, int in, int out_pad, int in_pad, __bf16* W, __bf16* Wt,
                    hipStream_t s) {
  const int n = out_pad * in_pad;
  hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, s, master, out, in, out_pad, in_pad, W, Wt);
  return hipGetLastError();
}

}  // namespace pmc
