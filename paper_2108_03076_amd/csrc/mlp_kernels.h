// Launchers of the surrogate MLP kernels (BF16 MFMA GEMMs and helpers).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pmc {

// C [M x N] FP32 (split-K: `splits` partial products, C[z][M][ldc]) = A Bt^T.
hipError_t mlp_gemm_f32(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb, int splits,
                        float* C, int ldc, hipStream_t s);
// Hidden layer forward with saved pre-activations Z, H = gelu(Z) and H^T.
hipError_t mlp_gemm_hidden(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb,
                           const float* bias, float* Z, __bf16* H, __bf16* Ht, hipStream_t s);
// Hidden layer forward for inference (H only).
hipError_t mlp_gemm_hidden_infer(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb,
                                 const float* bias, __bf16* H, hipStream_t s);
// Output layer: y[row] = ((A Bt^T)[row][0] + bias[0]) * scale.
hipError_t mlp_gemm_out(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb, const float* bias,
                        float* y, float scale, hipStream_t s);
// Back-propagation through a hidden layer: dZ = (A Bt^T) * gelu'(Z), and dZ^T.
hipError_t mlp_gemm_back_hidden(int M, int N, int K, const __bf16* A, int lda, const __bf16* Bt, int ldb,
                                const float* Z, __bf16* dZ, __bf16* dZt, hipStream_t s);
hipError_t mlp_scale_inputs(const float* x, int n, int n_in, const float* lo, const float* hi, int B, __bf16* X,
                            __bf16* Xt, hipStream_t s);
hipError_t mlp_loss(const float* yhat, const float* t, int n, int B, float inv_scale, float grad_scale, __bf16* dZ,
                    __bf16* dZt, double* part, double* acc, hipStream_t s);
hipError_t mlp_reduce_splits(const float* partial, int splits, size_t zstride, int ldp, int rows, int cols,
                             float* g, hipStream_t s);
hipError_t mlp_rowsum(const __bf16* dZt, int B, int rows, float* g, hipStream_t s);
hipError_t mlp_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s);
hipError_t mlp_pack(const float* master, int out, int in, int out_pad, int in_pad, __bf16* W, __bf16* Wt,
                    hipStream_t s);
// Fused inference of the width-256 network for n samples: y[i] = price of
// row i of x [n][n_in] (lohi: the input box, lo[0..31] then hi[0..31]; W1
// [256][16], W2 and W3 [256][256], W4 [32][256] padded BF16 weights; b*
// FP32 biases).
hipError_t mlp_infer256(const float* x, int n, int n_in, const float* lohi, const __bf16* W1, const float* b1,
                        const __bf16* W2, const float* b2, const __bf16* W3, const float* b3, const __bf16* W4,
                        const float* b4, float y_scale, float* y, hipStream_t s);

}  // namespace pmc
