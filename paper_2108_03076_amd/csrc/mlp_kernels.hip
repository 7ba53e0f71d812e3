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

// Position of weight (o, k) of a layer with in_pad inputs in the
// fragment-ordered copy the fused inference reads: the 16-byte A-operand
// fragment of output tile o/32 at k step k/16 that lane o%32 + 32 ((k%16)/8)
// supplies, fragments stored one after another (tile-major, then k step),
// so a wave's fragment load reads 1 KB of consecutive bytes.
__device__ __forceinline__ size_t frag_index(int o, int k, int in_pad) {
  const int ks = in_pad / 16;
  const int f = (o >> 5) * ks + (k >> 4);
  const int lane = (o & 31) + 32 * ((k & 15) >> 3);
  return ((size_t)f * 64 + lane) * 8 + (k & 7);
}

// GELU in the tanh form of Hendrycks and Gimpel,
// gelu(z) = z/2 (1 + tanh(u)), u = sqrt(2/pi) (z + 0.044715 z^3),
// evaluated as z * sigma(2u) = z / (1 + 2^(z (A + B z^2))) with
// A = -2 sqrt(2/pi) log2(e), B = 0.044715 A: two multiplies, an FMA, an
// add, exp2 and a reciprocal.  For z -> -inf the exponential overflows to
// +inf and the result is -0; for z -> +inf it is z.
constexpr float kGeluA = -2.302208198144325f;
constexpr float kGeluB = -0.1029432395800235f;
__device__ __forceinline__ float gelu_sigma(float z) {
  const float v = fmaf(z * z, kGeluB, kGeluA) * z;
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(v));
}
__device__ __forceinline__ float gelu(float z) { return z * gelu_sigma(z); }
// d/dz of z sigma(2u): sigma + z sigma (1 - sigma) 2u'(z),
// 2u' = 2 sqrt(2/pi) (1 + 3 * 0.044715 z^2).
__device__ __forceinline__ float gelu_grad(float z) {
  const float r = gelu_sigma(z);
  const float du = fmaf(z * z, 0.21406444881780073f, 1.5957691216057308f);
  return fmaf(z * r * (1.0f - r), du, r);
}

// C = A * Bt^T with A [M x K] and Bt [N x K] row-major BF16 (K contiguous).
// Block (bx, by, bz) of the grid (N/64, M/64, splits): 4 waves on a 64 x 64
// output tile, each wave one 32 x 32 MFMA tile; bz selects the K chunk of
// k_chunk.  M, N multiples of 32, K and k_chunk multiples of 16, lda/ldb
// multiples of 8 (16-byte rows).
// MFMA operand layout (32x32x16): lane l supplies row l%32 of A (and of Bt)
// at k = 8*(l/32) .. +7; accumulator element e of lane l is
// C[8*(e/4) + 4*(l/32) + e%4][l%32].
// The block stages its 64 rows of A and of Bt through LDS, 64 k at a time
// in two alternating buffers: a thread loads two 16-byte pieces of each
// (rows t/8 and t/8 + 32, k offset 8 (t%8)), so one wave load reads eight
// whole rows of 128 bytes; read directly, each lane's own row made every
// load touch 32 cache lines, and the vector-memory pipeline bound the
// kernel.  The loads of four stages are issued together.  The products run in the same k order as before.  An epilogue
// with a transposed BF16 output (Epi::kTransposed) returns each element's
// transposed value; the wave stages its 32 x 32 tile in LDS as
// [column][row] and writes each column's 32 rows as one 64-byte segment.
// lds: kGemmLds elements.  Every wave of the block takes part in the loads
// and barriers; a wave outside the matrix skips the products.
constexpr int kTld = 40;              // staged output tile row: 32 rows + 8 padding
constexpr int kSld = 72;              // staged operand row: 64 k + 8 padding
constexpr int kStage = 64 * kSld;     // one operand's stage
constexpr int kGemmLds = 4 * kStage;  // A and Bt, two stages each: 36,864 bytes
template <class Epi>
__device__ __forceinline__ void gemm_nt_block(int M, int N, int K, const __bf16* __restrict__ A, int lda,
                                              const __bf16* __restrict__ Bt, int ldb, int k_chunk, const Epi& epi,
                                              int bx, int by, int bz, __bf16* lds) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int mb = by * 64, nb = bx * 64;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int m0 = mb + wm, n0 = nb + wn;
  const bool active = m0 < M && n0 < N;
  const int kbeg = bz * k_chunk;
  const int kend = min(K, kbeg + k_chunk);
  const int r = lane & 31, kh = (lane >> 5) * 8;
  // this thread's pieces of a stage
  const int lr = t >> 3, lk = (t & 7) * 8;
  const bool a0 = mb + lr < M, a1 = mb + lr + 32 < M, b0 = nb + lr < N, b1 = nb + lr + 32 < N;
  const __bf16* ga = A + (size_t)(mb + lr) * lda + lk;
  const __bf16* gb = Bt + (size_t)(nb + lr) * ldb + lk;
  // up to four stages (256 k) in flight at once: one memory latency per
  // 256 k rather than one per stage
  bf16x8 ra[4][2], rb[4][2];
  f32x16 acc;
  const float c0 = active ? epi.init(n0 + r) : 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = c0;
  for (int k0 = kbeg; k0 < kend; k0 += 256) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bf16x8 z;
#pragma unroll
      for (int j = 0; j < 8; ++j) z[j] = to_bf16(0.0f);
      const int k = k0 + 64 * q;
      const bool in = k + lk < kend;
      ra[q][0] = (in && a0) ? *reinterpret_cast<const bf16x8*>(ga + k) : z;
      ra[q][1] = (in && a1) ? *reinterpret_cast<const bf16x8*>(ga + (size_t)32 * lda + k) : z;
      rb[q][0] = (in && b0) ? *reinterpret_cast<const bf16x8*>(gb + k) : z;
      rb[q][1] = (in && b1) ? *reinterpret_cast<const bf16x8*>(gb + (size_t)32 * ldb + k) : z;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 64 * q;
      if (k >= kend) break;
      // stage q goes to buffer q % 2, last read two stages ago (before the
      // previous stage's barrier)
      __bf16* as = lds + (q & 1) * 2 * kStage;
      __bf16* bs = as + kStage;
      *reinterpret_cast<bf16x8*>(as + lr * kSld + lk) = ra[q][0];
      *reinterpret_cast<bf16x8*>(as + (lr + 32) * kSld + lk) = ra[q][1];
      *reinterpret_cast<bf16x8*>(bs + lr * kSld + lk) = rb[q][0];
      *reinterpret_cast<bf16x8*>(bs + (lr + 32) * kSld + lk) = rb[q][1];
      __syncthreads();
      if (active) {
        const __bf16* pa = as + (wm + r) * kSld + kh;
        const __bf16* pb = bs + (wn + r) * kSld + kh;
        const int steps = min(4, (kend - k) / 16);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (u < steps)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8*>(pa + 16 * u),
                                                          *reinterpret_cast<const bf16x8*>(pb + 16 * u), acc, 0,
                                                          0, 0);
      }
    }
  }
  // every wave's products are done before the staging area is reused
  __syncthreads();
  if (!active) return;
  const int col = n0 + r;
  if constexpr (Epi::kTransposed) {
    __bf16* tt = lds + w * 32 * kTld;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rl = 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      tt[r * kTld + rl] = epi(m0 + rl, col, acc[e], bz);
    }
    // the wave reads back what its lanes wrote (the fence orders the LDS
    // stores before the loads); lane l copies rows 16 (l%2) .. +15 of tile
    // column l/2
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int c = lane >> 1, h = (lane & 1) * 16;
    const bf16x8 v0 = *reinterpret_cast<const bf16x8*>(tt + c * kTld + h);
    const bf16x8 v1 = *reinterpret_cast<const bf16x8*>(tt + c * kTld + h + 8);
    epi.store_t(n0 + c, m0 + h, v0, v1);
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = m0 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      epi(row, col, acc[e], bz);
    }
  }
}

template <class Epi>
__global__ __launch_bounds__(256) void k_gemm_nt(int M, int N, int K, const __bf16* __restrict__ A, int lda,
                                                 const __bf16* __restrict__ Bt, int ldb, int k_chunk, Epi epi) {
  __shared__ __bf16 lds[kGemmLds];
  gemm_nt_block(M, N, K, A, lda, Bt, ldb, k_chunk, epi, (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, lds);
}

// Each epilogue also names the accumulators' starting value for an output
// column: the layer's bias (the matrix cores add the products to it), or 0.
struct EpiF32 {          // C[z][row][col] (split-K partials or plain output)
  static constexpr bool kTransposed = false;
  float* c; int ldc; size_t zstride;
  __device__ float init(int) const { return 0.0f; }
  __device__ void operator()(int row, int col, float v, int z) const { c[z * zstride + (size_t)row * ldc + col] = v; }
};

struct EpiHidden {       // z = b + v; Z = z; H = gelu(z) (BF16) and its transpose
  static constexpr bool kTransposed = true;
  const float* bias; float* Z; int ldz; __bf16* H; int ldh; __bf16* Ht; int ldht;
  __device__ float init(int col) const { return bias[col]; }
  __device__ __bf16 operator()(int row, int col, float z, int) const {
    Z[(size_t)row * ldz + col] = z;
    const __bf16 h = to_bf16(gelu(z));
    H[(size_t)row * ldh + col] = h;
    return h;
  }
  // Ht[col][row .. row + 15]
  __device__ void store_t(int col, int row, bf16x8 v0, bf16x8 v1) const {
    bf16x8* p = reinterpret_cast<bf16x8*>(Ht + (size_t)col * ldht + row);
    p[0] = v0;
    p[1] = v1;
  }
};

struct EpiHiddenInfer {  // H = gelu(b + v) (BF16) only
  static constexpr bool kTransposed = false;
  const float* bias; __bf16* H; int ldh;
  __device__ float init(int col) const { return bias[col]; }
  __device__ void operator()(int row, int col, float z, int) const {
    H[(size_t)row * ldh + col] = to_bf16(gelu(z));
  }
};

struct EpiOut {          // y = (b + v) * scale for output column 0
  static constexpr bool kTransposed = false;
  const float* bias; float* y; float scale;
  __device__ float init(int col) const { return col == 0 ? bias[0] : 0.0f; }
  __device__ void operator()(int row, int col, float v, int) const {
    if (col == 0) y[row] = v * scale;
  }
};

// Output layer of a training step: yhat = b + v for output column 0 into y,
// and the output gradient d = grad_scale (yhat - t inv_scale) (0 for rows
// >= n, t the targets or the step record's batch) as column 0 of dZ
// [rows][32] and row 0 of dZt [32][B], every other element of both 0.
struct EpiOutTrain {
  static constexpr bool kTransposed = true;
  const float* bias; float* y; const float* t; const TrainStep* ts; int n, B; float inv_scale, grad_scale;
  __bf16* dZ; __bf16* dZt;
  __device__ float init(int col) const { return col == 0 ? bias[0] : 0.0f; }
  __device__ __bf16 operator()(int row, int col, float v, int) const {
    float d = 0.0f;
    if (col == 0) {
      y[row] = v;
      if (row < n) {
        const float* tt = ts ? ts->y + ts->step * (int64_t)B : t;
        const float e = v - tt[row] * inv_scale;
        d = grad_scale * e;
      }
    }
    const __bf16 b = to_bf16(d);
    dZ[(size_t)row * 32 + col] = b;
    return b;
  }
  // dZt[col][row .. row + 15]
  __device__ void store_t(int col, int row, bf16x8 v0, bf16x8 v1) const {
    bf16x8* p = reinterpret_cast<bf16x8*>(dZt + (size_t)col * B + row);
    p[0] = v0;
    p[1] = v1;
  }
};

struct EpiBackHidden {   // dZ = dH * gelu'(Z) (BF16) and its transpose
  static constexpr bool kTransposed = true;
  const float* Z; int ldz; __bf16* dZ; int lddz; __bf16* dZt; int lddzt;
  __device__ float init(int) const { return 0.0f; }
  // dZt[col][row .. row + 15]
  __device__ void store_t(int col, int row, bf16x8 v0, bf16x8 v1) const {
    bf16x8* p = reinterpret_cast<bf16x8*>(dZt + (size_t)col * lddzt + row);
    p[0] = v0;
    p[1] = v1;
  }
  __device__ __bf16 operator()(int row, int col, float v, int) const {
    const float g = v * gelu_grad(Z[(size_t)row * ldz + col]);
    const __bf16 b = to_bf16(g);
    dZ[(size_t)row * lddz + col] = b;
    return b;
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
// With a step record, x is its batch of the current step instead.
__device__ __forceinline__ void scale_row(const float* __restrict__ x, int n, int n_in, const float* __restrict__ lo,
                                          const float* __restrict__ hi, int B, __bf16* __restrict__ X,
                                          __bf16* __restrict__ Xt, int i) {
  bf16x8 row[2];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    float v = 0.0f;
    if (i < n && j < n_in) v = 2.0f * (x[(size_t)i * n_in + j] - lo[j]) / (hi[j] - lo[j]) - 1.0f;
    const __bf16 b = to_bf16(v);
    if (j < 16) row[j >> 3][j & 7] = b;
    Xt[(size_t)j * B + i] = b;
  }
  bf16x8* px = reinterpret_cast<bf16x8*>(X + (size_t)i * 16);
  px[0] = row[0];
  px[1] = row[1];
}
__global__ void k_scale_inputs(const float* __restrict__ x, int n, int n_in, const float* __restrict__ lo,
                               const float* __restrict__ hi, int B, __bf16* __restrict__ X,
                               __bf16* __restrict__ Xt, const TrainStep* __restrict__ ts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  if (ts) x = ts->x + ts->step * (int64_t)B * n_in;
  scale_row(x, n, n_in, lo, hi, B, X, Xt, i);
}

// out[0] += sum of part[0..n) in a fixed order (one thread).
__global__ void k_sum_parts(const double* part, int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  out[0] += s;
}

// Row sums of dZt [rows_b][B] into gb: block bid covers rows 4 bid .. + 3,
// one wave per row (lane l sums elements 8 (l + 64 i) .. + 7 for i = 0, 1,
// .. with 16-byte loads, B a multiple of 8; then a butterfly).
__device__ __forceinline__ void bias_rows_block(const __bf16* __restrict__ dZt, int B, int rows_b,
                                                float* __restrict__ gb, int bid) {
  const int lane = threadIdx.x & 63;
  const int r = bid * 4 + (threadIdx.x >> 6);
  if (r >= rows_b) return;
  const __bf16* p = dZt + (size_t)r * B;
  float sum = 0.0f;
  for (int b = 8 * lane; b < B; b += 512) {
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(p + b);
#pragma unroll
    for (int j = 0; j < 8; ++j) sum += from_bf16(v[j]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
  if (lane == 0) gb[r] = sum;
}

// The weight and bias gradients of one layer in one launch.  Blocks
// [0, n_red) reduce the split-K partials: g[row][col] (rows < rows_real,
// cols < cols_real, row-major with ld cols_real) = the sum over the SPLITS
// partials partial[z][row][col] (ld ldp) in z order from 0.  The other
// blocks sum the rows of dZt (BF16 [rows_b][B]) into gb.  With a step
// record, block 0 also advances it: this launch is the last of a step's
// gradients, and nothing in it reads the record.
template <int SPLITS>
__device__ __forceinline__ void layer_grads_block(const float* __restrict__ partial, size_t zstride, int ldp,
                                                  int rows_real, int cols_real, float* __restrict__ g,
                                                  const __bf16* __restrict__ dZt, int B, int rows_b,
                                                  float* __restrict__ gb, int n_red, int bid) {
  if (bid < n_red) {
    const int i = bid * 256 + (int)threadIdx.x;
    if (i >= rows_real * cols_real) return;
    const int row = i / cols_real, col = i % cols_real;
    const float* p = partial + (size_t)row * ldp + col;
    float v[SPLITS];
#pragma unroll
    for (int z = 0; z < SPLITS; ++z) v[z] = p[z * zstride];
    float sum = 0.0f;
#pragma unroll
    for (int z = 0; z < SPLITS; ++z) sum += v[z];
    g[i] = sum;
    return;
  }
  bias_rows_block(dZt, B, rows_b, gb, bid - n_red);
}
template <int SPLITS>
__global__ __launch_bounds__(256) void k_layer_grads(const float* __restrict__ partial, size_t zstride, int ldp,
                                                     int rows_real, int cols_real, float* __restrict__ g,
                                                     const __bf16* __restrict__ dZt, int B, int rows_b,
                                                     float* __restrict__ gb, int n_red, TrainStep* ts_next) {
  if (ts_next && blockIdx.x == 0 && threadIdx.x == 0) ts_next->step += 1;
  layer_grads_block<SPLITS>(partial, zstride, ldp, rows_real, cols_real, g, dZt, B, rows_b, gb, n_red,
                            (int)blockIdx.x);
}

// The squared errors of a training batch summed per block of 256 rows,
// (yhat - t inv_scale)^2 in FP64 for rows < n, by a fixed tree over the
// block: part[(ts ? step * blocks : 0) + block].
struct LossGrid {
  const float* y; const float* t; const TrainStep* ts; int n, B; float inv_scale; double* part; int blocks;
};
__device__ __forceinline__ void loss_part_block(const LossGrid& lj, int bid, double* red) {
  const int i = bid * 256 + (int)threadIdx.x;
  double l = 0.0;
  if (i < lj.B && i < lj.n) {
    const float* tt = lj.ts ? lj.ts->y + lj.ts->step * (int64_t)lj.B : lj.t;
    const float e = lj.y[i] - tt[i] * lj.inv_scale;
    l = (double)e * (double)e;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lj.part[(lj.ts ? lj.ts->step * (int64_t)lj.blocks : 0) + bid] = red[0];
}

// A backward launch's jobs over one flat grid: blocks [0, nb) the
// back-propagation GEMM, then nw blocks of the weight-gradient GEMM, then
// the reduction's blocks, then those of one more layer's bias sums (a
// count of 0 leaves a job out), then those of the loss partials; the
// reduction's first block advances the step record when one is given.  The
// jobs share no outputs, and no block waits on another (a block's barriers
// are its own, every thread of it on the same job).
struct GemmGrid {
  int M, N, K; const __bf16* A; int lda; const __bf16* Bt; int ldb; int k_chunk; int gx, gy, gz;
  __device__ int blocks() const { return gx * gy * gz; }
};
struct RedGrid {
  const float* partial; size_t zstride; int ldp, rows, cols; float* g; const __bf16* dZt; int B, rows_b;
  float* gb; int n_red, blocks;
  const __bf16* dZt2; int rows_b2; float* gb2; int blocks2;   // one more layer's bias sums
  TrainStep* ts_next;
};
__global__ __launch_bounds__(256) void k_backward_step(GemmGrid bj, EpiBackHidden be, GemmGrid wj, EpiF32 we,
                                                       RedGrid rj, LossGrid lj) {
  __shared__ __bf16 lds[kGemmLds];
  int b = blockIdx.x;
  const int nb = bj.blocks();
  if (b < nb) {
    gemm_nt_block(bj.M, bj.N, bj.K, bj.A, bj.lda, bj.Bt, bj.ldb, bj.k_chunk, be, b % bj.gx, (b / bj.gx) % bj.gy,
                  b / (bj.gx * bj.gy), lds);
    return;
  }
  b -= nb;
  const int nw = wj.blocks();
  if (b < nw) {
    gemm_nt_block(wj.M, wj.N, wj.K, wj.A, wj.lda, wj.Bt, wj.ldb, wj.k_chunk, we, b % wj.gx, (b / wj.gx) % wj.gy,
                  b / (wj.gx * wj.gy), lds);
    return;
  }
  b -= nw;
  if (b < rj.blocks) {
    if (rj.ts_next && b == 0 && threadIdx.x == 0) rj.ts_next->step += 1;
    layer_grads_block<16>(rj.partial, rj.zstride, rj.ldp, rj.rows, rj.cols, rj.g, rj.dZt, rj.B, rj.rows_b, rj.gb,
                          rj.n_red, b);
    return;
  }
  b -= rj.blocks;
  if (b < rj.blocks2) {
    bias_rows_block(rj.dZt2, rj.B, rj.rows_b2, rj.gb2, b);
    return;
  }
  b -= rj.blocks2;
  if (b < lj.blocks) loss_part_block(lj, b, reinterpret_cast<double*>(lds));
}

// One Adam step on the FP32 master parameters followed by the BF16 copies
// W [out_pad][in_pad], Wt [in_pad][out_pad] and Wf (fragment order) of
// each updated weight (the zero padding is written once, at creation).
// With a step record, the learning rate and the bias corrections are its
// entries for the step whose gradients these are: the gradient launch has
// already advanced the record, so that step is step - 1.
__global__ void k_adam_pack(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2, MlpLayers L, const TrainStep* __restrict__ ts,
                            const float* __restrict__ part1, size_t zstride1, int ldp1, MlpNextInputs next,
                            int adam_blocks) {
  if ((int)blockIdx.x >= adam_blocks) {
    // the next step's scaled inputs (the record has advanced to it), if
    // the pass has one
    const int r = ((int)blockIdx.x - adam_blocks) * (int)blockDim.x + (int)threadIdx.x;
    if (r < next.B && ts->step < ts->n_steps)
      scale_row(ts->x + ts->step * (int64_t)next.B * next.n_in, next.B, next.n_in, next.lo, next.hi, next.B, next.X,
                next.Xt, r);
    return;
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (ts) {
    const float* h = ts->hyper + 3 * (ts->step - 1);
    lr = h[0]; c1 = h[1]; c2 = h[2];
  }
  float gi;
  if (part1 && i >= L.oW[0] && i < L.ob[0]) {
    // layer 1's weight gradient from its split-K partials, summed in z
    // order from 0 as the reduction of the other layers sums them
    const int64_t j = i - L.oW[0];
    const float* p = part1 + (size_t)(j / L.in[0]) * ldp1 + (j % L.in[0]);
    float pv[16];
#pragma unroll
    for (int z = 0; z < 16; ++z) pv[z] = p[z * zstride1];
    gi = 0.0f;
#pragma unroll
    for (int z = 0; z < 16; ++z) gi += pv[z];
  } else {
    gi = g[i];
  }
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
#pragma unroll
  for (int l = 0; l < 4; ++l)
    if (i >= L.oW[l] && i < L.ob[l]) {
      const int64_t j = i - L.oW[l];
      const int o = (int)(j / L.in[l]), k = (int)(j % L.in[l]);
      const __bf16 b = to_bf16(wi);
      L.W[l][(size_t)o * L.inp[l] + k] = b;
      L.Wt[l][(size_t)k * L.outp[l] + o] = b;
      L.Wf[l][frag_index(o, k, L.inp[l])] = b;
    }
}

// BF16 working copies of a layer's weights from the FP32 master [out][in]:
// W [out_pad][in_pad], Wt [in_pad][out_pad] and the fragment-ordered Wf,
// zero padded.
__global__ void k_pack(const float* __restrict__ master, int out, int in, int out_pad, int in_pad, __bf16* W,
                       __bf16* Wt, __bf16* Wf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= out_pad * in_pad) return;
  const int o = i / in_pad, k = i % in_pad;
  const float x = (o < out && k < in) ? master[(size_t)o * in + k] : 0.0f;
  const __bf16 b = to_bf16(x);
  W[(size_t)o * in_pad + k] = b;
  Wt[(size_t)k * out_pad + o] = b;
  Wf[frag_index(o, k, in_pad)] = b;
}

// Fused inference for width 256: a block carries 64 samples through the
// four layers with their BF16 activations in LDS, in two buffers (a layer
// reads one and writes the other, so one barrier per layer suffices; rows
// padded by 8 elements): 67.6 KB, so two blocks share a CU.  The matrix
// cores compute C^T = W X^T: operand A is a weight fragment (rows = output
// features), operand B an activation fragment (rows = samples), so a lane's
// accumulator holds four consecutive features of one sample (elements
// 4q .. 4q + 3 are features 8q + 4 (lane / 32) + 0..3 of the tile, sample
// lane % 32), which GELU turns into one 8-byte LDS store.  The accumulators
// start at the bias, as in the per-layer kernels, whose outputs these are
// bit for bit.  A block has eight waves; wave w owns features 32w .. 32w + 31
// (one feature tile) of every layer and holds their weights in registers
// (64 of its 124 vector registers) for both 32-sample tiles, so four waves
// share each SIMD and one's matrix products overlap another's GELU; within
// a wave, the GELU of the first sample tile is interleaved with the
// products of the second.  (Four waves per block, each holding two feature
// tiles' weights in 242 registers, ran two waves per SIMD: 3-4 % slower.)
constexpr int kInferRows = 64;
constexpr int kInferW = 256;
constexpr int kInferLd = kInferW + 8;
constexpr int kInferThreads = 512;
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void bias_init(f32x16& acc, const float* __restrict__ b) {
  const int h4 = 4 * ((threadIdx.x & 63) >> 5);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = *reinterpret_cast<const float4*>(b + 8 * q + h4);
    acc[4 * q + 0] = v.x; acc[4 * q + 1] = v.y; acc[4 * q + 2] = v.z; acc[4 * q + 3] = v.w;
  }
}

// This wave's weight fragments of a layer with K = 16 KS inputs, k steps
// K0 .. K1 - 1, from the fragment-ordered copy Wf: output tile w (features
// 32w ..), one 1 KB wave load per k step.  With OUT set, the layer is the
// output layer (one 32-row tile, loaded by every wave).
template <int KS, int K0 = 0, int K1 = KS, bool OUT = false>
__device__ __forceinline__ void load_weights(bf16x8 (&wf)[16], const __bf16* __restrict__ Wf) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = K0; k < K1; ++k)
    wf[k] = *reinterpret_cast<const bf16x8*>(Wf + ((size_t)((OUT ? 0 : w) * KS + k) * 64 + lane) * 8);
}

// GELU of accumulator elements 4q .. 4q + 3 of one tile into the lane's
// sample row (dst: that row at the tile's first feature + 4 (lane / 32)).
__device__ __forceinline__ void gelu_quad(const f32x16& acc, int q, __bf16* dst) {
  bf16x4 v;
  v[0] = to_bf16(gelu(acc[4 * q + 0]));
  v[1] = to_bf16(gelu(acc[4 * q + 1]));
  v[2] = to_bf16(gelu(acc[4 * q + 2]));
  v[3] = to_bf16(gelu(acc[4 * q + 3]));
  *reinterpret_cast<bf16x4*>(dst + 8 * q) = v;
}

// A training forward also keeps each hidden layer's pre-activations Z
// (FP32 [B][256]), activations H (BF16 [B][256]) and their transpose Ht
// (BF16 [256][B]) for the backward pass; g0 is the block's first sample.
struct LayerOut {
  float* Z; __bf16* H; __bf16* Ht; int64_t g0; int B;
};
// The quad's values as gelu_quad stores them, into the training outputs
// (sample `row` of the block, the tile's features f0 .. f0 + 3).
__device__ __forceinline__ void keep_quad(const f32x16& acc, int q, const LayerOut& to, int row, int f0) {
  const int64_t s = to.g0 + row;
  const int f = f0 + 8 * q;
  float4 z;
  z.x = acc[4 * q + 0]; z.y = acc[4 * q + 1]; z.z = acc[4 * q + 2]; z.w = acc[4 * q + 3];
  *reinterpret_cast<float4*>(to.Z + s * kInferW + f) = z;
  bf16x4 h;
  h[0] = to_bf16(gelu(z.x)); h[1] = to_bf16(gelu(z.y)); h[2] = to_bf16(gelu(z.z)); h[3] = to_bf16(gelu(z.w));
  *reinterpret_cast<bf16x4*>(to.H + s * kInferW + f) = h;
#pragma unroll
  for (int i = 0; i < 4; ++i) to.Ht[(int64_t)(f + i) * to.B + s] = h[i];
}

// One hidden layer (K = 16 KS inputs, 256 outputs) for the block's 64
// samples: out = gelu(b + W in).  The products of sample tile 1 are
// written interleaved with the GELU of tile 0 (one quad per four k steps),
// so the matrix cores and the vector unit of a wave work at the same time;
// the next layer's weights are loaded into the weight registers once this
// layer's products are issued, half before and half after the GELU of
// tile 1 (their latency hides behind the GELU and the barrier).
template <int KS, int KSN, bool NEXT_OUT = false, bool TRAIN = false, int ST = 2>
__device__ __forceinline__ void hidden_layer(const __bf16* in, __bf16* out, bf16x8 (&wf)[16],
                                             const float* __restrict__ bl, const __bf16* __restrict__ Wnext,
                                             const LayerOut& to = LayerOut{}) {
  const int lane = threadIdx.x & 63, r = lane & 31, kh = (lane >> 5) * 8, w = threadIdx.x >> 6;
  const int h4 = 4 * (lane >> 5);
  f32x16 acc[2];   // [sample tile]
#pragma unroll
  for (int st = 0; st < ST; ++st) bias_init(acc[st], bl + 32 * w);
  if constexpr (ST == 1) {   // one sample tile: products, then GELU
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(in + r * kInferLd + 16 * k + kh);
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[k], b, acc[0], 0, 0, 0);
    }
    load_weights<KSN, 0, KSN / 2, NEXT_OUT>(wf, Wnext);
    __bf16* o0 = out + r * kInferLd + 32 * w + h4;
#pragma unroll
    for (int q = 0; q < 4; ++q) gelu_quad(acc[0], q, o0);
    if constexpr (TRAIN) {
#pragma unroll
      for (int q = 0; q < 4; ++q) keep_quad(acc[0], q, to, r, 32 * w + h4);
    }
    load_weights<KSN, KSN / 2, KSN, NEXT_OUT>(wf, Wnext);
    return;
  }
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(in + r * kInferLd + 16 * k + kh);
    acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[k], b, acc[0], 0, 0, 0);
  }
  __bf16* o0 = out + r * kInferLd + 32 * w + h4;
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(in + (32 + r) * kInferLd + 16 * k + kh);
    acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[k], b, acc[1], 0, 0, 0);
    if (KS == 16 && (k & 3) == 0) gelu_quad(acc[0], k >> 2, o0);
  }
  if (KS != 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) gelu_quad(acc[0], q, o0);
  }
  if constexpr (TRAIN) {
#pragma unroll
    for (int q = 0; q < 4; ++q) keep_quad(acc[0], q, to, r, 32 * w + h4);
  }
  load_weights<KSN, 0, KSN / 2, NEXT_OUT>(wf, Wnext);
  __bf16* o1 = out + (32 + r) * kInferLd + 32 * w + h4;
#pragma unroll
  for (int q = 0; q < 4; ++q) gelu_quad(acc[1], q, o1);
  if constexpr (TRAIN) {
#pragma unroll
    for (int q = 0; q < 4; ++q) keep_quad(acc[1], q, to, 32 + r, 32 * w + h4);
  }
  load_weights<KSN, KSN / 2, KSN, NEXT_OUT>(wf, Wnext);
}

__global__ __launch_bounds__(kInferThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_mlp_infer256(
    const float* __restrict__ x, int n, int n_in, const float* __restrict__ lohi, const __bf16* __restrict__ W1,
    const float* __restrict__ b1, const __bf16* __restrict__ W2, const float* __restrict__ b2,
    const __bf16* __restrict__ W3, const float* __restrict__ b3, const __bf16* __restrict__ W4,
    const float* __restrict__ b4, float y_scale, float* __restrict__ y) {
  __shared__ __bf16 act[2][kInferRows * kInferLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 31, kh = (lane >> 5) * 8;
  const int64_t g0 = (int64_t)blockIdx.x * kInferRows;   // global row of the block's first row
  bf16x8 wf[16];
  load_weights<1>(wf, W1);
  if (threadIdx.x < 4 * kInferRows) {
    // scaled inputs in columns 0..15 (zero beyond n_in and beyond n):
    // thread t fills row t/4, columns 4 (t%4) ..
    const int row = threadIdx.x >> 2, j0 = 4 * (threadIdx.x & 3);
    const int64_t gi = g0 + row;
    bf16x4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float t = 0.0f;
      if (gi < n && j0 + j < n_in)
        t = 2.0f * (x[gi * n_in + j0 + j] - lohi[j0 + j]) / (lohi[32 + j0 + j] - lohi[j0 + j]) - 1.0f;
      v[j] = to_bf16(t);
    }
    *reinterpret_cast<bf16x4*>(&act[0][row * kInferLd + j0]) = v;
  }
  __syncthreads();
  hidden_layer<1, 16>(act[0], act[1], wf, b1, W2);
  __syncthreads();
  hidden_layer<16, 16>(act[1], act[0], wf, b2, W3);
  __syncthreads();
  // the output layer's fragments (W4: one 32-row tile, 16 k steps) are
  // loaded by every wave
  hidden_layer<16, 16, true>(act[0], act[1], wf, b3, W4);
  __syncthreads();
  if (w < 2) {   // waves 0 and 1: samples 32w .. 32w + 31; feature 0 is element 0 of lanes 0..31
    f32x16 out;
#pragma unroll
    for (int e = 0; e < 16; ++e) out[e] = 0.0f;
    if (lane < 32) out[0] = b4[0];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&act[1][(32 * w + r) * kInferLd + 16 * k + kh]);
      out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[k], b, out, 0, 0, 0);
    }
    if (lane < 32 && g0 + 32 * w + r < n) y[g0 + 32 * w + r] = out[0] * y_scale;
  }
}

// The forward pass of a training step for width 256 in one launch, as
// k_mlp_infer256 computes it (the same values bit for bit as the per-layer
// kernels): the block's 64 rows of the scaled inputs X [B][16] are read
// into LDS, each hidden layer also keeps Z, H and Ht (LayerOut), and the
// output layer writes yhat into y and the output gradient d = grad_scale
// (yhat - t inv_scale) (0 for rows >= n; t the targets or the step
// record's batch) as column 0 of dZ [B][32] and row 0 of dZt [32][B],
// every other element of both 0.
struct TrainFwd {
  const __bf16* X; float* Z[3]; __bf16* H[3]; __bf16* Ht[3]; float* y; const float* t; const TrainStep* ts;
  int n, B; float inv_scale, grad_scale; __bf16* dZ; __bf16* dZt;
};
// (A training batch of B samples is B / 64 blocks, far fewer than the
// CUs at the usual batch sizes: the kernel takes the registers it needs
// rather than the four waves per SIMD of inference, which spilled.)
constexpr int kTrainRows = 32;   // samples per block of the training forward (one sample tile)
__global__ __launch_bounds__(kInferThreads) __attribute__((amdgpu_waves_per_eu(2, 4))) void k_mlp_train_fwd256(
    TrainFwd a, const __bf16* __restrict__ W1, const float* __restrict__ b1, const __bf16* __restrict__ W2,
    const float* __restrict__ b2, const __bf16* __restrict__ W3, const float* __restrict__ b3,
    const __bf16* __restrict__ W4, const float* __restrict__ b4) {
  __shared__ __bf16 act[2][kTrainRows * kInferLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 31, kh = (lane >> 5) * 8;
  const int64_t g0 = (int64_t)blockIdx.x * kTrainRows;
  bf16x8 wf[16];
  load_weights<1>(wf, W1);
  if (threadIdx.x < 2 * kTrainRows) {   // row t/2, columns 8 (t%2) ..
    const int row = threadIdx.x >> 1, c = 8 * (threadIdx.x & 1);
    *reinterpret_cast<bf16x8*>(&act[0][row * kInferLd + c]) =
        *reinterpret_cast<const bf16x8*>(a.X + (g0 + row) * 16 + c);
  }
  __syncthreads();
  hidden_layer<1, 16, false, true, 1>(act[0], act[1], wf, b1, W2, LayerOut{a.Z[0], a.H[0], a.Ht[0], g0, a.B});
  __syncthreads();
  hidden_layer<16, 16, false, true, 1>(act[1], act[0], wf, b2, W3, LayerOut{a.Z[1], a.H[1], a.Ht[1], g0, a.B});
  __syncthreads();
  hidden_layer<16, 16, true, true, 1>(act[0], act[1], wf, b3, W4, LayerOut{a.Z[2], a.H[2], a.Ht[2], g0, a.B});
  __syncthreads();
  if (w < 1) {   // wave 0: the block's 32 samples; feature 0 is element 0 of lanes 0..31
    f32x16 out;
#pragma unroll
    for (int e = 0; e < 16; ++e) out[e] = 0.0f;
    if (lane < 32) out[0] = b4[0];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&act[1][(32 * w + r) * kInferLd + 16 * k + kh]);
      out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[k], b, out, 0, 0, 0);
    }
    if (lane < 32) {
      const int64_t row = g0 + 32 * w + r;
      const float v = out[0];
      a.y[row] = v;
      float d = 0.0f;
      if (row < a.n) {
        const float* tt = a.ts ? a.ts->y + a.ts->step * (int64_t)a.B : a.t;
        const float e = v - tt[row] * a.inv_scale;
        d = a.grad_scale * e;
      }
      const __bf16 db = to_bf16(d);
      bf16x8 first, zero;
#pragma unroll
      for (int j = 0; j < 8; ++j) { first[j] = to_bf16(0.0f); zero[j] = to_bf16(0.0f); }
      first[0] = db;
      bf16x8* pz = reinterpret_cast<bf16x8*>(a.dZ + row * 32);
      pz[0] = first; pz[1] = zero; pz[2] = zero; pz[3] = zero;
#pragma unroll
      for (int j = 0; j < 32; ++j) a.dZt[(int64_t)j * a.B + row] = j == 0 ? db : to_bf16(0.0f);
    }
  }
}

}  // namespace

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
hipError_t mlp_scale_inputs(const float* x, int n, int n_in, const float* lo, const float* hi, int B, __bf16* X,
                            __bf16* Xt, const TrainStep* ts, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inputs, dim3((B + 255) / 256), dim3(256), 0, s, x, n, n_in, lo, hi, B, X, Xt, ts);
  return hipGetLastError();
}
hipError_t mlp_gemm_out_train(int M, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb, const float* bias,
                              float* y, const float* t, int n, float inv_scale, float grad_scale, __bf16* dZ,
                              __bf16* dZt, const TrainStep* ts, hipStream_t s) {
  if (!ts && !t) return hipErrorInvalidValue;
  return gemm(M, 32, K, A, lda, Bt, ldb, 1, EpiOutTrain{bias, y, t, ts, n, M, inv_scale, grad_scale, dZ, dZt}, s);
}
hipError_t mlp_sum_parts(const double* part, int64_t n, double* acc, hipStream_t s) {
  if (n < 1 || n > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part, (int)n, acc);
  return hipGetLastError();
}
hipError_t mlp_layer_grads(const float* partial, int splits, size_t zstride, int ldp, int rows, int cols, float* g,
                           const __bf16* dZt, int B, int rows_b, float* gb, TrainStep* ts_next, hipStream_t s) {
  if (splits != 16 || B % 8 || rows < 1 || cols < 1 || rows_b < 0) return hipErrorInvalidValue;
  const int n_red = (rows * cols + 255) / 256;
  hipLaunchKernelGGL(k_layer_grads<16>, dim3(n_red + (rows_b + 3) / 4), dim3(256), 0, s, partial, zstride, ldp, rows,
                     cols, g, dZt, B, rows_b, gb, n_red, ts_next);
  return hipGetLastError();
}
namespace {
// The grid of one GEMM job (validated as gemm() does); a job with M = 0
// gets no blocks.
bool gemm_grid(const MlpGemmJob& j, int splits, GemmGrid& g) {
  g = GemmGrid{j.M, j.N, j.K, j.A, j.lda, j.Bt, j.ldb, 0, 0, 0, 0};
  if (j.M == 0) return true;
  if (j.M < 0 || j.N < 1 || j.K < 16 || j.M % 32 || j.N % 32 || j.K % 16 || j.lda % 8 || j.ldb % 8 || splits < 1 ||
      !j.A || !j.Bt)
    return false;
  int chunk = (j.K + splits - 1) / splits;
  chunk = (chunk + 15) / 16 * 16;
  g.k_chunk = chunk;
  g.gx = (j.N + 63) / 64;
  g.gy = (j.M + 63) / 64;
  g.gz = splits;
  return true;
}
}  // namespace

hipError_t mlp_backward_step(const MlpGemmJob& back, const float* Z, __bf16* dZ, __bf16* dZt,
                             const MlpGemmJob& wgrad, int splits, float* wpart, int ldc, const MlpGradJob& red,
                             const MlpLossJob& loss, hipStream_t s) {
  GemmGrid bj, wj;
  if (!gemm_grid(back, 1, bj) || !gemm_grid(wgrad, splits, wj)) return hipErrorInvalidValue;
  if (back.M && (!Z || !dZ || !dZt)) return hipErrorInvalidValue;
  if (wgrad.M && (!wpart || ldc < wgrad.N)) return hipErrorInvalidValue;
  RedGrid rj{red.partial, red.zstride, red.ldp, red.rows, red.cols, red.g, red.dZt, red.B, red.rows_b, red.gb, 0, 0,
             red.dZt2, red.rows_b2, red.gb2, 0, red.ts_next};
  if (red.rows) {
    if (red.rows < 1 || red.cols < 1 || red.rows_b < 1 || red.B % 8 || !red.partial || !red.g || !red.dZt || !red.gb)
      return hipErrorInvalidValue;
    rj.n_red = (red.rows * red.cols + 255) / 256;
    rj.blocks = rj.n_red + (red.rows_b + 3) / 4;
    if (red.rows_b2) {
      if (red.rows_b2 < 0 || !red.dZt2 || !red.gb2) return hipErrorInvalidValue;
      rj.blocks2 = (red.rows_b2 + 3) / 4;
    }
  } else if (red.rows_b2 || red.ts_next) {
    return hipErrorInvalidValue;
  }
  LossGrid lj{loss.y, loss.t, loss.ts, loss.n, loss.B, loss.inv_scale, loss.part, 0};
  if (loss.B) {
    if (loss.B < 1 || loss.n < 0 || !loss.y || !loss.part || (!loss.t && !loss.ts)) return hipErrorInvalidValue;
    lj.blocks = (loss.B + 255) / 256;
  }
  const int64_t total = (int64_t)bj.gx * bj.gy * bj.gz + (int64_t)wj.gx * wj.gy * wj.gz + rj.blocks + rj.blocks2 +
                        lj.blocks;
  if (total < 1 || total > INT32_MAX) return hipErrorInvalidValue;
  const EpiBackHidden be{Z, back.N, dZ, back.N, dZt, back.M};
  const EpiF32 we{wpart, ldc, (size_t)wgrad.M * ldc};
  hipLaunchKernelGGL(k_backward_step, dim3((unsigned)total), dim3(256), 0, s, bj, be, wj, we, rj, lj);
  return hipGetLastError();
}
hipError_t mlp_adam_pack(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                         float eps, float c1, float c2, const MlpLayers& L, const TrainStep* ts,
                         const float* part1, size_t zstride1, int ldp1, const MlpNextInputs* next, hipStream_t s) {
  if (next && (!ts || next->B < 1 || next->n_in < 1 || next->n_in > 16)) return hipErrorInvalidValue;
  const int adam_blocks = (int)((n + 255) / 256);
  const int scale_blocks = next ? (next->B + 255) / 256 : 0;
  hipLaunchKernelGGL(k_adam_pack, dim3((unsigned)(adam_blocks + scale_blocks)), dim3(256), 0, s, w, m, v, g, n, lr,
                     b1, b2, eps, c1, c2, L, ts, part1, zstride1, ldp1, next ? *next : MlpNextInputs{}, adam_blocks);
  return hipGetLastError();
}
hipError_t mlp_infer256(const float* x, int n, int n_in, const float* lohi, const __bf16* W1, const float* b1,
                        const __bf16* W2, const float* b2, const __bf16* W3, const float* b3, const __bf16* W4,
                        const float* b4, float y_scale, float* y, hipStream_t s) {
  if (n < 1 || n_in < 1 || n_in > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_infer256, dim3((n + kInferRows - 1) / kInferRows), dim3(kInferThreads), 0, s, x, n, n_in,
                     lohi, W1, b1, W2, b2, W3, b3, W4, b4, y_scale, y);
  return hipGetLastError();
}
hipError_t mlp_train_forward256(const __bf16* X, float* const Z[3], __bf16* const H[3], __bf16* const Ht[3],
                                const __bf16* W1, const float* b1, const __bf16* W2, const float* b2,
                                const __bf16* W3, const float* b3, const __bf16* W4, const float* b4, float* y,
                                const float* t, int n, int B, float inv_scale, float grad_scale, __bf16* dZ,
                                __bf16* dZt, const TrainStep* ts, hipStream_t s) {
  if (B < kTrainRows || B % kTrainRows || n < 0 || n > B || (!t && !ts)) return hipErrorInvalidValue;
  TrainFwd a{X, {Z[0], Z[1], Z[2]}, {H[0], H[1], H[2]}, {Ht[0], Ht[1], Ht[2]}, y, t, ts, n, B, inv_scale, grad_scale,
             dZ, dZt};
  hipLaunchKernelGGL(k_mlp_train_fwd256, dim3(B / kTrainRows), dim3(kInferThreads), 0, s, a, W1, b1, W2, b2, W3, b3,
                     W4, b4);
  return hipGetLastError();
}
hipError_t mlp_pack(const float* master, int out, int in, int out_pad, int in_pad, __bf16* W, __bf16* Wt,
                    __bf16* Wf, hipStream_t s) {
  if (out_pad % 32 || in_pad % 16) return hipErrorInvalidValue;
  const int n = out_pad * in_pad;
  hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, s, master, out, in, out_pad, in_pad, W, Wt, Wf);
  return hipGetLastError();
}

}  // namespace pmc
