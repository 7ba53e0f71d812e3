// Launchers of the surrogate MLP kernels (BF16 MFMA GEMMs and helpers).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pmc {

// Where a captured training step finds what changes from step to step:
// the epoch's inputs and targets (batch `step` of B rows each) and the
// per-step learning rate and Adam bias corrections (hyper[3 * step + 0..2]).
// Device memory; the last kernel of a step increments `step`.
struct TrainStep {
  const float* x;
  const float* y;
  const float* hyper;
  int64_t step;
  int64_t n_steps;   // steps of the pass (the inputs of step n_steps do not exist)
};
// The scaled inputs of a training step's batch (X [B][16], Xt [32][B]
// BF16, as mlp_scale_inputs makes them): with it, the Adam launch also
// makes those of the step that follows (the step record has advanced),
// if the pass has one.
struct MlpNextInputs {
  const float* lo = nullptr; const float* hi = nullptr; int n_in = 0, B = 0;
  __bf16* X = nullptr; __bf16* Xt = nullptr;
};

// The four layers' places in the flat parameter vector and their BF16
// copies (for the fused Adam and repack).
struct MlpLayers {
  int64_t oW[4], ob[4];
  int out[4], in[4], outp[4], inp[4];
  __bf16* W[4];
  __bf16* Wt[4];
  __bf16* Wf[4];   // fragment-ordered copies (fused inference)
};

// Hidden layer forward with saved pre-activations Z, H = gelu(Z) and H^T.
hipError_t mlp_gemm_hidden(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb,
                           const float* bias, float* Z, __bf16* H, __bf16* Ht, hipStream_t s);
// Hidden layer forward for inference (H only).
hipError_t mlp_gemm_hidden_infer(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb,
                                 const float* bias, __bf16* H, hipStream_t s);
// Output layer: y[row] = ((A Bt^T)[row][0] + bias[0]) * scale.
hipError_t mlp_gemm_out(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb, const float* bias,
                        float* y, float scale, hipStream_t s);
// x raw inputs [n][n_in] (or, with ts, the step record's batch).
hipError_t mlp_scale_inputs(const float* x, int n, int n_in, const float* lo, const float* hi, int B, __bf16* X,
                            __bf16* Xt, const TrainStep* ts, hipStream_t s);
// Output layer of a training step (N = 32 padded outputs, column 0 real):
// yhat = bias[0] + (A Bt^T)[row][0] into y [M], and the output gradient
// d = grad_scale (yhat - t inv_scale) (0 for rows >= n) as column 0 of dZ
// [M][32] and row 0 of dZt [32][M], every other element of both 0; t the
// targets [n] or, with ts, the step record's batch.
hipError_t mlp_gemm_out_train(int M, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb, const float* bias,
                              float* y, const float* t, int n, float inv_scale, float grad_scale, __bf16* dZ,
                              __bf16* dZt, const TrainStep* ts, hipStream_t s);
// Adds part[0 .. n) in order to acc[0] (one thread).
hipError_t mlp_sum_parts(const double* part, int64_t n, double* acc, hipStream_t s);
// One layer's weight gradient g [rows][cols] from its 16 split-K partials
// and bias gradient gb [rows_b] (row sums of dZt [rows_b][B]; rows_b = 0:
// none) in one launch; with ts_next, the launch also advances the step
// record.
hipError_t mlp_layer_grads(const float* partial, int splits, size_t zstride, int ldp, int rows, int cols, float* g,
                           const __bf16* dZt, int B, int rows_b, float* gb, TrainStep* ts_next, hipStream_t s);
// One launch of the backward pass that runs up to four independent jobs
// side by side (a job with no rows is left out):
//  * back: back-propagation to the layer below, dZ = (A Bt^T) * gelu'(Z)
//    (BF16 [M][N]) and dZ^T ([N][M]), Z FP32 [M][N];
//  * wgrad: a layer's weight gradient A Bt^T as `splits` partial products
//    over chunks of K, into wpart [splits][M][ldc];
//  * red: another layer's weight and bias gradients from its partials, as
//    mlp_layer_grads (its step record advanced by its first block);
//  * loss: the batch's loss partials (MlpLossJob below).
// The jobs must not share outputs: red reads a partials buffer that wgrad
// does not write; no job reads another job's output.
struct MlpGemmJob {
  int M = 0, N = 0, K = 0;
  const __bf16* A = nullptr; int lda = 0;
  const __bf16* Bt = nullptr; int ldb = 0;
};
struct MlpGradJob {
  const float* partial = nullptr; size_t zstride = 0; int ldp = 0, rows = 0, cols = 0;
  float* g = nullptr;
  const __bf16* dZt = nullptr; int B = 0, rows_b = 0;
  float* gb = nullptr;
  // optional: the bias gradient gb2 [rows_b2] of one more layer (row sums
  // of dZt2 [rows_b2][B]), and the step record to advance
  const __bf16* dZt2 = nullptr; int rows_b2 = 0;
  float* gb2 = nullptr;
  TrainStep* ts_next = nullptr;
};
// loss: the batch's squared errors of the scaled targets, (y - t
// inv_scale)^2 for rows < n in FP64, summed per block of 256 rows into
// part[(ts ? step * blocks : 0) + block] (B = 0: no such job).
struct MlpLossJob {
  const float* y = nullptr; const float* t = nullptr; const TrainStep* ts = nullptr;
  int n = 0, B = 0; float inv_scale = 1.0f; double* part = nullptr;
};
hipError_t mlp_backward_step(const MlpGemmJob& back, const float* Z, __bf16* dZ, __bf16* dZt,
                             const MlpGemmJob& wgrad, int splits, float* wpart, int ldc, const MlpGradJob& red,
                             const MlpLossJob& loss, hipStream_t s);
// Adam on the FP32 master parameters and the BF16 repack of the weights
// (with ts: lr, c1, c2 from its current step).  With part1, the gradient of
// layer 1's weights is the sum of its 16 split-K partials (part1
// [16][rows][ldp1], zstride1 apart), taken here in the order
// mlp_layer_grads takes it, instead of g.
hipError_t mlp_adam_pack(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                         float eps, float c1, float c2, const MlpLayers& L, const TrainStep* ts,
                         const float* part1, size_t zstride1, int ldp1, const MlpNextInputs* next, hipStream_t s);
// The forward pass of a training step for width 256 in one launch (B a
// multiple of 32): from the scaled inputs X [B][16] the hidden layers'
// Z (FP32 [B][256]), H (BF16 [B][256]) and Ht (BF16 [256][B]), yhat into
// y [B] and the output gradient as mlp_gemm_out_train writes it, with the
// fragment-ordered weights Wf (W1..W4) and FP32 biases; the same values bit
// for bit as the per-layer kernels.
hipError_t mlp_train_forward256(const __bf16* X, float* const Z[3], __bf16* const H[3], __bf16* const Ht[3],
                                const __bf16* W1, const float* b1, const __bf16* W2, const float* b2,
                                const __bf16* W3, const float* b3, const __bf16* W4, const float* b4, float* y,
                                const float* t, int n, int B, float inv_scale, float grad_scale, __bf16* dZ,
                                __bf16* dZt, const TrainStep* ts, hipStream_t s);
// W [out_pad][in_pad], Wt [in_pad][out_pad] and the fragment-ordered Wf
// (A-operand fragments of 32-row output tiles and 16-wide k steps, each
// 64 lanes x 16 bytes, tile-major) from the FP32 master weights.
hipError_t mlp_pack(const float* master, int out, int in, int out_pad, int in_pad, __bf16* W, __bf16* Wt,
                    __bf16* Wf, hipStream_t s);
// Fused inference of the width-256 network for n samples: y[i] = price of
// row i of x [n][n_in] (lohi: the input box, lo[0..31] then hi[0..31]; W1
// [256][16], W2 and W3 [256][256], W4 [32][256] padded BF16 weights in
// fragment order (mlp_pack's Wf); b* FP32 biases).
hipError_t mlp_infer256(const float* x, int n, int n_in, const float* lohi, const __bf16* W1, const float* b1,
                        const __bf16* W2, const float* b2, const __bf16* W3, const float* b3, const __bf16* W4,
                        const float* b4, float y_scale, float* y, hipStream_t s);

}  // namespace pmc
