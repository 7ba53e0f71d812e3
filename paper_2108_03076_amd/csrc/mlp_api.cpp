// C ABI of the learned surrogate: an MLP n_in -> W -> W -> W -> 1 with GELU,
// BF16 weights and activations, FP32 accumulation on the matrix cores, FP32
// master weights and Adam.  Parameters are kept flat on the device in the
// order W1 b1 W2 b2 W3 b3 W4 b4 (each W row-major [out][in]).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pmc.h"
#include "ctx.h"
#include "mlp_kernels.h"

using namespace pmc;

namespace {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
  ~Buf() { if (p) (void)hipFree(p); }
  hipError_t ensure(size_t n) {
    if (n <= cap) return hipSuccess;
    if (p) { (void)hipFree(p); p = nullptr; cap = 0; }
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) cap = n;
    return e;
  }
  template <typename T> T* as() const { return (T*)p; }
};

constexpr int kSplits = 16;   // split-K factor of the weight-gradient GEMMs

}  // namespace

struct pmc_mlp {
  pmc_ctx* ctx = nullptr;
  int n_in = 8, width = 256;
  double y_scale = 100.0;
  std::vector<double> lo, hi;   // the input box (host copy, for saving)
  int64_t n_params = 0;
  int64_t step = 0;
  // flat parameter offsets
  int64_t oW[4], ob[4];
  int out_[4], in_[4], outp[4], inp[4];
  Buf master, m, v, grad, lohi;
  Buf W[4], Wt[4], Wf[4];
  // batch-sized work buffers
  int B = 0;
  // partial[2]: split-K weight-gradient partials, alternating between
  // layers so that one layer's reduction runs beside the next one's products
  Buf X, Xt, Z[3], H[3], Ht[3], Y, dZ4, dZ4t, dZ[3], dZt[3], part_loss, loss_acc, partial[2];
  Buf px, py;   // surrogate pricing: the in-box points and their predictions
  int64_t gen = 0;   // bumped whenever a work buffer moves (a captured step is then stale)
  // kGraphSteps training steps captured as a graph (batch size B_graph,
  // buffers of generation gen_graph)
  Buf tstep, hyper, part_epoch;   // the step record, per-step hyper-parameters, per-step loss partials
  std::vector<float> hyper_host;
  TrainStep tstep_host{};
  hipGraphExec_t step_exec = nullptr;
  hipStream_t capture = nullptr;   // set while a step is being captured
  int B_graph = 0;
  int64_t gen_graph = -1;
  double adam_graph[3] = {-1, -1, -1};   // beta1, beta2, eps the captured step was made with
  ~pmc_mlp() { if (step_exec) (void)hipGraphExecDestroy(step_exec); }
  MlpLayers layers() {
    MlpLayers L;
    for (int l = 0; l < 4; ++l) {
      L.oW[l] = oW[l]; L.ob[l] = ob[l]; L.out[l] = out_[l]; L.in[l] = in_[l]; L.outp[l] = outp[l];
      L.inp[l] = inp[l]; L.W[l] = W[l].as<__bf16>(); L.Wt[l] = Wt[l].as<__bf16>(); L.Wf[l] = Wf[l].as<__bf16>();
    }
    return L;
  }
};

#define MLP_TRY(m, expr)                                                                           \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return ctx_fail((m)->ctx, e_ == hipErrorOutOfMemory ? PMC_E_OOM : PMC_E_HIP,                 \
                      std::string(#expr) + ": " + hipGetErrorString(e_));                          \
  } while (0)

namespace {

// The stream the surrogate's work goes to: the context's, or while a
// training step is captured the capturing stream.
hipStream_t stream_of(const pmc_mlp* M) { return M->capture ? M->capture : ctx_stream(M->ctx); }

int pack_all(pmc_mlp* M) {
  hipStream_t s = stream_of(M);
  for (int l = 0; l < 4; ++l)
    MLP_TRY(M, mlp_pack(M->master.as<float>() + M->oW[l], M->out_[l], M->in_[l], M->outp[l], M->inp[l],
                        M->W[l].as<__bf16>(), M->Wt[l].as<__bf16>(), M->Wf[l].as<__bf16>(), s));
  return PMC_OK;
}

int ensure_batch(pmc_mlp* M, int B) {
  if (B <= M->B) return PMC_OK;
  const int W = M->width;
  const size_t b = (size_t)B;
  MLP_TRY(M, M->X.ensure(b * 16 * 2));
  MLP_TRY(M, M->Xt.ensure(b * 32 * 2));
  for (int l = 0; l < 3; ++l) {
    MLP_TRY(M, M->Z[l].ensure(b * W * 4));
    MLP_TRY(M, M->H[l].ensure(b * W * 2));
    MLP_TRY(M, M->Ht[l].ensure(b * W * 2));
    MLP_TRY(M, M->dZ[l].ensure(b * W * 2));
    MLP_TRY(M, M->dZt[l].ensure(b * W * 2));
  }
  MLP_TRY(M, M->Y.ensure(b * 4));
  MLP_TRY(M, M->dZ4.ensure(b * 32 * 2));
  MLP_TRY(M, M->dZ4t.ensure(b * 32 * 2));
  MLP_TRY(M, M->part_loss.ensure(((b + 255) / 256) * 8));
  MLP_TRY(M, M->loss_acc.ensure(8));
  for (auto& p : M->partial) MLP_TRY(M, p.ensure((size_t)kSplits * W * W * 4));
  M->B = B;
  M->gen++;
  return PMC_OK;
}

// Forward pass over B rows (n real) of raw inputs x (with ts: the step
// record's batch); saves what backward needs when train is set.
int forward(pmc_mlp* M, const float* x, int n, int B, bool train, const TrainStep* ts = nullptr,
            const float* y = nullptr) {
  hipStream_t s = stream_of(M);
  const int W = M->width;
  const float* w = M->master.as<float>();
  if (train && W == 256) {
    // one launch: the hidden layers (with Z, H, H^T) and the output layer
    // with its loss gradient, from the scaled inputs
    if (!ts)
      MLP_TRY(M, mlp_scale_inputs(x, n, M->n_in, M->lohi.as<float>(), M->lohi.as<float>() + 32, B,
                                  M->X.as<__bf16>(), M->Xt.as<__bf16>(), nullptr, s));
    float* const Z[3] = {M->Z[0].as<float>(), M->Z[1].as<float>(), M->Z[2].as<float>()};
    __bf16* const H[3] = {M->H[0].as<__bf16>(), M->H[1].as<__bf16>(), M->H[2].as<__bf16>()};
    __bf16* const Ht[3] = {M->Ht[0].as<__bf16>(), M->Ht[1].as<__bf16>(), M->Ht[2].as<__bf16>()};
    MLP_TRY(M, mlp_train_forward256(M->X.as<__bf16>(), Z, H, Ht, M->Wf[0].as<__bf16>(), w + M->ob[0],
                                    M->Wf[1].as<__bf16>(), w + M->ob[1], M->Wf[2].as<__bf16>(), w + M->ob[2],
                                    M->Wf[3].as<__bf16>(), w + M->ob[3], M->Y.as<float>(), y, n, B,
                                    (float)(1.0 / M->y_scale), 2.0f / (float)n, M->dZ4.as<__bf16>(),
                                    M->dZ4t.as<__bf16>(), ts, s));
    return PMC_OK;
  }
  // (a training step's inputs were scaled by the previous step's Adam
  // launch, or at the start of the pass)
  if (!ts)
    MLP_TRY(M, mlp_scale_inputs(x, n, M->n_in, M->lohi.as<float>(), M->lohi.as<float>() + 32, B,
                                M->X.as<__bf16>(), M->Xt.as<__bf16>(), nullptr, s));
  const __bf16* in = M->X.as<__bf16>();
  int ld = 16;
  for (int l = 0; l < 3; ++l) {
    if (train)
      MLP_TRY(M, mlp_gemm_hidden(B, W, M->inp[l], in, ld, M->W[l].as<__bf16>(), M->inp[l], w + M->ob[l],
                                 M->Z[l].as<float>(), M->H[l].as<__bf16>(), M->Ht[l].as<__bf16>(), s));
    else
      MLP_TRY(M, mlp_gemm_hidden_infer(B, W, M->inp[l], in, ld, M->W[l].as<__bf16>(), M->inp[l], w + M->ob[l],
                                       M->H[l].as<__bf16>(), s));
    in = M->H[l].as<__bf16>();
    ld = W;
  }
  // (a training step's output layer runs with its loss gradient, first in
  // backward())
  if (!train)
    MLP_TRY(M, mlp_gemm_out(B, 32, W, in, W, M->W[3].as<__bf16>(), W, w + M->ob[3], M->Y.as<float>(),
                            (float)M->y_scale, s));
  return PMC_OK;
}

// Loss and gradients (into M->grad) of mean((yhat - y/y_scale)^2) over n
// rows.  Without a step record: targets y, and the batch's sum of squared
// errors is added to loss_acc.  With one (a training step): its batch, the
// loss partials go to the pass's slots (part_epoch), and the last gradient
// launch advances the record.
int backward(pmc_mlp* M, const float* y, int n, int B, TrainStep* ts = nullptr) {
  hipStream_t s = stream_of(M);
  const int W = M->width;
  float* g = M->grad.as<float>();
  const float inv_scale = (float)(1.0 / M->y_scale);
  // output layer: yhat, and its gradient dZ4 = 2 (yhat - y / y_scale) / n
  // (width 256: done by the forward launch)
  if (W != 256)
    MLP_TRY(M, mlp_gemm_out_train(B, W, M->H[2].as<__bf16>(), W, M->W[3].as<__bf16>(), W,
                                M->master.as<float>() + M->ob[3], M->Y.as<float>(), y, n, inv_scale, 2.0f / (float)n,
                                M->dZ4.as<__bf16>(), M->dZ4t.as<__bf16>(), ts, s));
  MlpLossJob loss;
  loss.y = M->Y.as<float>();
  loss.t = y;
  loss.ts = ts;
  loss.n = n;
  loss.B = B;
  loss.inv_scale = inv_scale;
  loss.part = ts ? M->part_epoch.as<double>() : M->part_loss.as<double>();
  // Four launches after the output layer.  Each back-propagates to the
  // layer below (`back`, but the last), forms the split-K weight-gradient
  // partials of the layer whose dZ it reads (`wgrad`) and reduces the
  // previous launch's partials with that layer's bias sums (`red`, but the
  // first); the partials alternate between two buffers.  The first also
  // sums the batch's loss partials; the last also sums layer 1's bias
  // gradient and advances the step record (the loss partials have read
  // it); layer 1's weight partials are summed by Adam in a training step
  // (in the same order), and by one more launch otherwise.
  float* pa = M->partial[0].as<float>();
  float* pb = M->partial[1].as<float>();
  const MlpGemmJob none;
  const MlpGradJob no_red;
  const MlpLossJob no_loss;
  // layer 4: dW4 partials (dZ4^T H3), dZ3 = (dZ4 W4) * gelu'(Z3)
  MLP_TRY(M, mlp_backward_step(MlpGemmJob{B, W, 32, M->dZ4.as<__bf16>(), 32, M->Wt[3].as<__bf16>(), 32},
                               M->Z[2].as<float>(), M->dZ[2].as<__bf16>(), M->dZt[2].as<__bf16>(),
                               MlpGemmJob{32, W, B, M->dZ4t.as<__bf16>(), B, M->Ht[2].as<__bf16>(), B}, kSplits, pa,
                               W, no_red, loss, s));
  // without a step record: the batch's squared errors go to loss_acc
  if (!ts) MLP_TRY(M, mlp_sum_parts(M->part_loss.as<double>(), (B + 255) / 256, M->loss_acc.as<double>(), s));
  // layer 3 and dZ2; dW4 and db4
  MLP_TRY(M, mlp_backward_step(MlpGemmJob{B, W, W, M->dZ[2].as<__bf16>(), W, M->Wt[2].as<__bf16>(), W},
                               M->Z[1].as<float>(), M->dZ[1].as<__bf16>(), M->dZt[1].as<__bf16>(),
                               MlpGemmJob{W, W, B, M->dZt[2].as<__bf16>(), B, M->Ht[1].as<__bf16>(), B}, kSplits, pb,
                               W, MlpGradJob{pa, (size_t)32 * W, W, 1, W, g + M->oW[3], M->dZ4t.as<__bf16>(), B, 1,
                                             g + M->ob[3]},
                               no_loss, s));
  // layer 2 and dZ1; dW3 and db3
  MLP_TRY(M, mlp_backward_step(MlpGemmJob{B, W, W, M->dZ[1].as<__bf16>(), W, M->Wt[1].as<__bf16>(), W},
                               M->Z[0].as<float>(), M->dZ[0].as<__bf16>(), M->dZt[0].as<__bf16>(),
                               MlpGemmJob{W, W, B, M->dZt[1].as<__bf16>(), B, M->Ht[0].as<__bf16>(), B}, kSplits, pa,
                               W, MlpGradJob{pb, (size_t)W * W, W, W, W, g + M->oW[2], M->dZt[2].as<__bf16>(), B, W,
                                             g + M->ob[2]},
                               no_loss, s));
  // layer 1 (X^T has 32 padded rows); dW2 and db2; db1; the step record
  // advances (the loss has read it)
  MlpGradJob red2{pa, (size_t)W * W, W, W, W, g + M->oW[1], M->dZt[1].as<__bf16>(), B, W, g + M->ob[1]};
  red2.dZt2 = M->dZt[0].as<__bf16>();
  red2.rows_b2 = W;
  red2.gb2 = g + M->ob[0];
  red2.ts_next = ts;
  MLP_TRY(M, mlp_backward_step(none, nullptr, nullptr, nullptr,
                               MlpGemmJob{W, 32, B, M->dZt[0].as<__bf16>(), B, M->Xt.as<__bf16>(), B}, kSplits, pb,
                               32, red2, no_loss, s));
  // dW1: in a training step, Adam sums its partials itself; otherwise here
  if (!ts)
    MLP_TRY(M, mlp_layer_grads(pb, kSplits, (size_t)W * 32, 32, W, M->n_in, g + M->oW[0], nullptr, B, 0, nullptr,
                               nullptr, s));
  return PMC_OK;
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" int pmc_mlp_create(pmc_ctx* ctx, int n_in, int width, uint64_t seed, const double* in_lo,
                              const double* in_hi, double y_scale, pmc_mlp** out) {
  if (!ctx || !out || !in_lo || !in_hi) return PMC_E_ARG;
  if (n_in < 1 || n_in > 16 || width < 32 || width % 32 || width > 1024 || !(y_scale > 0))
    return ctx_fail(ctx, PMC_E_UNSUPPORTED, "surrogate needs 1 <= n_in <= 16 and width a multiple of 32 up to 1024");
  for (int i = 0; i < n_in; ++i)
    if (!std::isfinite(in_lo[i]) || !std::isfinite(in_hi[i]) || !(in_hi[i] > in_lo[i]))
      return ctx_fail(ctx, PMC_E_ARG, "input box must be finite with hi > lo");
  auto M = std::make_unique<pmc_mlp>();
  M->ctx = ctx;
  M->n_in = n_in;
  M->width = width;
  M->y_scale = y_scale;
  M->lo.assign(in_lo, in_lo + n_in);
  M->hi.assign(in_hi, in_hi + n_in);
  const int W = width;
  const int outs[4] = {W, W, W, 1}, ins[4] = {n_in, W, W, W};
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    M->out_[l] = outs[l];
    M->in_[l] = ins[l];
    M->outp[l] = l == 3 ? 32 : W;
    M->inp[l] = l == 0 ? 16 : W;
    M->oW[l] = off;
    off += (int64_t)outs[l] * ins[l];
    M->ob[l] = off;
    off += outs[l];
  }
  M->n_params = off;
  // PyTorch-style initialisation: U(-1/sqrt(in), 1/sqrt(in)) for W and b
  std::vector<float> h((size_t)off);
  uint64_t st = seed;
  for (int l = 0; l < 4; ++l) {
    const double a = 1.0 / std::sqrt((double)ins[l]);
    for (int64_t i = M->oW[l]; i < M->ob[l] + outs[l]; ++i) {
      const double u = (double)(splitmix(st) >> 11) * 0x1p-53;
      h[i] = (float)((2.0 * u - 1.0) * a);
    }
  }
  std::vector<float> lohi(64, 0.0f);
  for (int i = 0; i < n_in; ++i) { lohi[i] = (float)in_lo[i]; lohi[32 + i] = (float)in_hi[i]; }
  for (int i = n_in; i < 32; ++i) { lohi[i] = 0.0f; lohi[32 + i] = 1.0f; }
  pmc_mlp* m = M.get();
  hipStream_t s = ctx_stream(ctx);
  MLP_TRY(m, hipSetDevice(ctx_device(ctx)));
  const size_t pb = (size_t)off * 4;
  MLP_TRY(m, m->master.ensure(pb));
  MLP_TRY(m, m->m.ensure(pb));
  MLP_TRY(m, m->v.ensure(pb));
  MLP_TRY(m, m->grad.ensure(pb));
  MLP_TRY(m, m->lohi.ensure(64 * 4));
  for (int l = 0; l < 4; ++l) {
    MLP_TRY(m, m->W[l].ensure((size_t)m->outp[l] * m->inp[l] * 2));
    MLP_TRY(m, m->Wt[l].ensure((size_t)m->outp[l] * m->inp[l] * 2));
    MLP_TRY(m, m->Wf[l].ensure((size_t)m->outp[l] * m->inp[l] * 2));
  }
  MLP_TRY(m, hipMemcpyAsync(m->master.p, h.data(), pb, hipMemcpyHostToDevice, s));
  MLP_TRY(m, hipMemsetAsync(m->m.p, 0, pb, s));
  MLP_TRY(m, hipMemsetAsync(m->v.p, 0, pb, s));
  MLP_TRY(m, hipMemcpyAsync(m->lohi.p, lohi.data(), 64 * 4, hipMemcpyHostToDevice, s));
  int rc = pack_all(m);
  if (rc != PMC_OK) return rc;
  MLP_TRY(m, hipStreamSynchronize(s));
  *out = M.release();
  return PMC_OK;
}

extern "C" void pmc_mlp_free(pmc_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(ctx_stream(m->ctx));
  delete m;
}

extern "C" int64_t pmc_mlp_num_params(const pmc_mlp* m) { return m ? m->n_params : -1; }

extern "C" int pmc_mlp_get_params(const pmc_mlp* m, float* out) {
  if (!m || !out) return PMC_E_ARG;
  pmc_mlp* M = const_cast<pmc_mlp*>(m);
  MLP_TRY(M, hipMemcpyAsync(out, m->master.p, (size_t)m->n_params * 4, hipMemcpyDeviceToHost, ctx_stream(m->ctx)));
  MLP_TRY(M, hipStreamSynchronize(ctx_stream(m->ctx)));
  return PMC_OK;
}

extern "C" int pmc_mlp_set_params(pmc_mlp* m, const float* in) {
  if (!m || !in) return PMC_E_ARG;
  hipStream_t s = ctx_stream(m->ctx);
  for (int64_t i = 0; i < m->n_params; ++i)
    if (!std::isfinite(in[i])) return ctx_fail(m->ctx, PMC_E_ARG, "parameters must be finite");
  MLP_TRY(m, hipMemcpyAsync(m->master.p, in, (size_t)m->n_params * 4, hipMemcpyHostToDevice, s));
  MLP_TRY(m, hipMemsetAsync(m->m.p, 0, (size_t)m->n_params * 4, s));
  MLP_TRY(m, hipMemsetAsync(m->v.p, 0, (size_t)m->n_params * 4, s));
  m->step = 0;
  int rc = pack_all(m);
  if (rc != PMC_OK) return rc;
  MLP_TRY(m, hipStreamSynchronize(s));
  return PMC_OK;
}

extern "C" int pmc_mlp_infer(pmc_mlp* m, const float* x, float* y, int64_t n) {
  if (!m || !x || !y || n < 1 || n > (1ll << 30)) return PMC_E_ARG;
  hipStream_t s = ctx_stream(m->ctx);
  // enqueued on the context's stream only: the caller orders its use of y
  // on that stream (or synchronizes)
  if (m->width == 256) {   // one fused kernel: all four layers per block of 64 samples
    const float* w = m->master.as<float>();
    const int chunk = 1 << 24;
    for (int64_t o = 0; o < n; o += chunk) {
      const int k = (int)std::min<int64_t>(chunk, n - o);
      MLP_TRY(m, mlp_infer256(x + o * m->n_in, k, m->n_in, m->lohi.as<float>(), m->Wf[0].as<__bf16>(), w + m->ob[0],
                              m->Wf[1].as<__bf16>(), w + m->ob[1], m->Wf[2].as<__bf16>(), w + m->ob[2],
                              m->Wf[3].as<__bf16>(), w + m->ob[3], (float)m->y_scale, y + o, s));
    }
    return PMC_OK;
  }
  const int chunk = 1 << 16;
  for (int64_t o = 0; o < n; o += chunk) {
    const int k = (int)std::min<int64_t>(chunk, n - o);
    const int B = (k + 63) / 64 * 64;
    int rc = ensure_batch(m, B);
    if (rc != PMC_OK) return rc;
    rc = forward(m, x + o * m->n_in, k, B, false);
    if (rc != PMC_OK) return rc;
    // the k real rows of the prices (network output times y_scale)
    MLP_TRY(m, hipMemcpyAsync(y + o, m->Y.p, (size_t)k * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  return PMC_OK;
}

extern "C" int pmc_mlp_loss_grad(pmc_mlp* m, const float* x, const float* y, int64_t n, double* loss,
                                 float* grad_out) {
  if (!m || !x || !y || !loss || !grad_out || n < 1 || n > (1 << 16)) return PMC_E_ARG;
  hipStream_t s = ctx_stream(m->ctx);
  const int B = (int)((n + 63) / 64 * 64);
  int rc = ensure_batch(m, B);
  if (rc != PMC_OK) return rc;
  MLP_TRY(m, hipMemsetAsync(m->loss_acc.p, 0, 8, s));
  rc = forward(m, x, (int)n, B, true, nullptr, y);
  if (rc == PMC_OK) rc = backward(m, y, (int)n, B);
  if (rc != PMC_OK) return rc;
  double acc = 0;
  MLP_TRY(m, hipMemcpyAsync(&acc, m->loss_acc.p, 8, hipMemcpyDeviceToHost, s));
  MLP_TRY(m, hipMemcpyAsync(grad_out, m->grad.p, (size_t)m->n_params * 4, hipMemcpyDeviceToHost, s));
  MLP_TRY(m, hipStreamSynchronize(s));
  *loss = acc / (double)n;
  return PMC_OK;
}

namespace {

// Learning rate (cosine schedule) and Adam bias corrections of Adam step
// number `step` (1-based), as the FP32 values the update uses; the moving
// averages use the FP32 betas, and so do their bias corrections.
void step_hyper(const pmc_train_opts* o, int64_t step, float out[3]) {
  const double frac = std::min(1.0, (double)(step - 1) / (double)o->total_steps);
  const double lr = o->lr_min + 0.5 * (o->lr_max - o->lr_min) * (1.0 + std::cos(M_PI * frac));
  const float b1 = (float)o->beta1, b2 = (float)o->beta2;
  out[0] = (float)lr;
  out[1] = (float)(1.0 - std::pow((double)b1, (double)step));
  out[2] = (float)(1.0 - std::pow((double)b2, (double)step));
}

// One training step over batch ts->step of the step record: forward, loss
// and gradients (whose last launch advances the record), then Adam with
// the BF16 repack.
int enqueue_step(pmc_mlp* M, const pmc_train_opts* o, int B, TrainStep* ts) {
  int rc = forward(M, nullptr, B, B, true, ts);
  if (rc == PMC_OK) rc = backward(M, nullptr, B, B, ts);
  if (rc != PMC_OK) return rc;
  hipStream_t s = stream_of(M);
  MlpNextInputs next;
  next.lo = M->lohi.as<float>();
  next.hi = M->lohi.as<float>() + 32;
  next.n_in = M->n_in;
  next.B = B;
  next.X = M->X.as<__bf16>();
  next.Xt = M->Xt.as<__bf16>();
  MLP_TRY(M, mlp_adam_pack(M->master.as<float>(), M->m.as<float>(), M->v.as<float>(), M->grad.as<float>(),
                           M->n_params, 0.0f, (float)o->beta1, (float)o->beta2, (float)o->eps, 1.0f, 1.0f,
                           M->layers(), ts, M->partial[1].as<float>(), (size_t)M->width * 32, 32, &next, s));
  return PMC_OK;
}

// kGraphSteps training steps captured as one graph for batch size B, the
// current work buffers and the Adam constants (betas, eps); captured again
// when any of them changes.  The batch position, the learning rate and the
// bias corrections come from the step record, so one graph serves every
// run of kGraphSteps steps of every epoch (the steps left over are issued
// one launch at a time).  No memset is captured.  (A graph of one step
// cost about 5 us per replay more than its launches issued one by one;
// with 16 steps per replay the two take the same time.)
constexpr int kGraphSteps = 16;
int step_graph(pmc_mlp* M, const pmc_train_opts* o, int B) {
  if (M->step_exec && M->B_graph == B && M->gen_graph == M->gen && M->adam_graph[0] == o->beta1 &&
      M->adam_graph[1] == o->beta2 && M->adam_graph[2] == o->eps)
    return PMC_OK;
  if (M->step_exec) { (void)hipGraphExecDestroy(M->step_exec); M->step_exec = nullptr; }
  hipStream_t cap = nullptr;
  MLP_TRY(M, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return ctx_fail(M->ctx, PMC_E_HIP, std::string("training step capture: ") + hipGetErrorString(e));
  }
  M->capture = cap;
  int rc = PMC_OK;
  for (int k = 0; k < kGraphSteps && rc == PMC_OK; ++k) rc = enqueue_step(M, o, B, M->tstep.as<TrainStep>());
  M->capture = nullptr;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cap, &graph);
  (void)hipStreamDestroy(cap);
  if (rc != PMC_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
  if (e != hipSuccess)
    return ctx_fail(M->ctx, PMC_E_HIP, std::string("training step capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&M->step_exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    M->step_exec = nullptr;
    return ctx_fail(M->ctx, PMC_E_HIP, std::string("training step graph: ") + hipGetErrorString(e));
  }
  M->B_graph = B;
  M->gen_graph = M->gen;
  M->adam_graph[0] = o->beta1; M->adam_graph[1] = o->beta2; M->adam_graph[2] = o->eps;
  return PMC_OK;
}

}  // namespace

extern "C" int pmc_mlp_train_epoch(pmc_mlp* m, const float* x, const float* y, int64_t n, const pmc_train_opts* o,
                                   double* mean_loss) {
  if (!m || !x || !y || !o || n < 1) return PMC_E_ARG;
  if (o->batch < 64 || o->batch % 64 || o->batch > (1 << 20) || o->total_steps < 1 || !(o->lr_max > 0) ||
      !(o->lr_min >= 0) || !(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1) || !(o->eps > 0) ||
      (o->eager != 0 && o->eager != 1))
    return ctx_fail(m->ctx, PMC_E_ARG, "bad training options (batch must be a multiple of 64)");
  hipStream_t s = ctx_stream(m->ctx);
  const int B = o->batch;
  const int64_t steps = n / B;   // full batches only
  if (steps < 1) return ctx_fail(m->ctx, PMC_E_ARG, "fewer samples than one batch");
  int rc = ensure_batch(m, B);
  if (rc != PMC_OK) return rc;
  // the step record of this epoch: its batches and each step's hyper-parameters
  MLP_TRY(m, hipSetDevice(ctx_device(m->ctx)));
  MLP_TRY(m, m->tstep.ensure(sizeof(TrainStep)));
  MLP_TRY(m, m->hyper.ensure((size_t)steps * 3 * sizeof(float)));
  const int64_t n_part = steps * ((B + 255) / 256);   // loss partials: one per step and loss block
  if ((size_t)n_part * sizeof(double) > m->part_epoch.cap) {
    MLP_TRY(m, m->part_epoch.ensure((size_t)n_part * sizeof(double)));
    m->gen++;   // a captured step writes its partials there
  }
  // the previous epoch's uploads must be done before their host copies change
  MLP_TRY(m, hipStreamSynchronize(s));
  m->hyper_host.resize((size_t)steps * 3);
  for (int64_t k = 0; k < steps; ++k) step_hyper(o, m->step + 1 + k, &m->hyper_host[(size_t)k * 3]);
  m->tstep_host = TrainStep{x, y, m->hyper.as<float>(), 0, steps};
  MLP_TRY(m, hipMemcpyAsync(m->hyper.p, m->hyper_host.data(), m->hyper_host.size() * sizeof(float),
                            hipMemcpyHostToDevice, s));
  MLP_TRY(m, hipMemcpyAsync(m->tstep.p, &m->tstep_host, sizeof(TrainStep), hipMemcpyHostToDevice, s));
  MLP_TRY(m, hipMemsetAsync(m->loss_acc.p, 0, 8, s));
  // the first step's scaled inputs (each step's Adam launch makes the next's)
  MLP_TRY(m, mlp_scale_inputs(nullptr, B, m->n_in, m->lohi.as<float>(), m->lohi.as<float>() + 32, B,
                              m->X.as<__bf16>(), m->Xt.as<__bf16>(), m->tstep.as<TrainStep>(), s));
  if (o->eager) {
    for (int64_t k = 0; k < steps; ++k) {
      rc = enqueue_step(m, o, B, m->tstep.as<TrainStep>());
      if (rc != PMC_OK) return rc;
    }
  } else {
    if (steps >= kGraphSteps) {
      rc = step_graph(m, o, B);
      if (rc != PMC_OK) return rc;
    }
    for (int64_t k = 0; k + kGraphSteps <= steps; k += kGraphSteps) MLP_TRY(m, hipGraphLaunch(m->step_exec, s));
    for (int64_t k = steps / kGraphSteps * kGraphSteps; k < steps; ++k) {
      rc = enqueue_step(m, o, B, m->tstep.as<TrainStep>());
      if (rc != PMC_OK) return rc;
    }
  }
  MLP_TRY(m, mlp_sum_parts(m->part_epoch.as<double>(), n_part, m->loss_acc.as<double>(), s));
  m->step += steps;
  double acc = 0;
  MLP_TRY(m, hipMemcpyAsync(&acc, m->loss_acc.p, 8, hipMemcpyDeviceToHost, s));
  MLP_TRY(m, hipStreamSynchronize(s));
  if (mean_loss) *mean_loss = acc / (double)(steps * B);
  return PMC_OK;
}

extern "C" int pmc_mlp_price(pmc_mlp* m, const double* x, int64_t n, const pmc_payoff* p, const pmc_batch* b,
                             const pmc_gbm* model, const pmc_opts* o, double* price_out, double* std_err_out,
                             int* route_out) {
  if (!m || !x || n < 1 || !p || !b || !model || !o || !price_out) return PMC_E_ARG;
  if (b->n_inst != n) return ctx_fail(m->ctx, PMC_E_ARG, "the batch must describe the n points, in order");
  pmc_payoff_info info;
  if (pmc_payoff_get_info(p, &info) != PMC_OK) return PMC_E_ARG;
  const int D = m->n_in, A = info.n_assets, nt = info.n_tvars, np = info.n_params;
  // route: inside the network's input box (every input within [lo, hi]) or not
  std::vector<int64_t> in_box, out_box;
  for (int64_t i = 0; i < n; ++i) {
    bool inside = true;
    for (int d = 0; d < D; ++d) {
      const double v = x[i * D + d];
      if (!(v >= m->lo[d] && v <= m->hi[d])) inside = false;   // NaN is outside
    }
    (inside ? in_box : out_box).push_back(i);
  }
  std::vector<double> price(n, 0.0), se(n, 0.0);
  hipStream_t s = ctx_stream(m->ctx);
  if (!in_box.empty()) {
    const int64_t k = (int64_t)in_box.size();
    std::vector<float> xs((size_t)k * D);
    for (int64_t j = 0; j < k; ++j)
      for (int d = 0; d < D; ++d) xs[(size_t)j * D + d] = (float)x[in_box[j] * D + d];
    MLP_TRY(m, hipSetDevice(ctx_device(m->ctx)));
    MLP_TRY(m, m->px.ensure(xs.size() * sizeof(float)));
    MLP_TRY(m, m->py.ensure((size_t)k * sizeof(float)));
    MLP_TRY(m, hipMemcpyAsync(m->px.p, xs.data(), xs.size() * sizeof(float), hipMemcpyHostToDevice, s));
    int rc = pmc_mlp_infer(m, m->px.as<float>(), m->py.as<float>(), k);
    if (rc != PMC_OK) return rc;
    std::vector<float> ys((size_t)k);
    MLP_TRY(m, hipMemcpyAsync(ys.data(), m->py.p, (size_t)k * sizeof(float), hipMemcpyDeviceToHost, s));
    MLP_TRY(m, hipStreamSynchronize(s));
    for (int64_t j = 0; j < k; ++j) price[in_box[j]] = ys[j];
  }
  if (!out_box.empty()) {
    // the out-of-box instances as one batch; each keeps its own stream id
    const size_t k = out_box.size();
    std::vector<int32_t> tenv(k * nt);
    std::vector<double> params(k * np), spot, vol, corr;
    std::vector<uint32_t> ids(k);
    if (nt && !b->tenv) return ctx_fail(m->ctx, PMC_E_ARG, "null tenv");
    if (np && !b->params) return ctx_fail(m->ctx, PMC_E_ARG, "null params");
    if (b->per_instance_model && (!b->spot || !b->vol)) return ctx_fail(m->ctx, PMC_E_ARG, "null spot or vol");
    for (size_t j = 0; j < k; ++j) {
      const int64_t i = out_box[j];
      for (int v = 0; v < nt; ++v) tenv[j * nt + v] = b->tenv[i * nt + v];
      for (int q = 0; q < np; ++q) params[j * np + q] = b->params[i * np + q];
      ids[j] = b->instance_ids ? b->instance_ids[i] : (uint32_t)i;
      if (b->per_instance_model) {
        spot.insert(spot.end(), b->spot + i * A, b->spot + (i + 1) * A);
        vol.insert(vol.end(), b->vol + i * A, b->vol + (i + 1) * A);
        if (b->corr) corr.insert(corr.end(), b->corr + i * A * A, b->corr + (i + 1) * A * A);
      }
    }
    pmc_batch sub{};
    sub.n_inst = (int)k;
    sub.tenv = nt ? tenv.data() : nullptr;
    sub.params = np ? params.data() : nullptr;
    sub.per_instance_model = b->per_instance_model;
    sub.spot = b->per_instance_model ? spot.data() : nullptr;
    sub.vol = b->per_instance_model ? vol.data() : nullptr;
    sub.corr = (b->per_instance_model && b->corr) ? corr.data() : nullptr;
    sub.instance_ids = ids.data();
    std::vector<pmc_result> res(k);
    int rc = pmc_price_batch(m->ctx, p, &sub, model, o, res.data());
    if (rc != PMC_OK) return rc;
    for (size_t j = 0; j < k; ++j) {
      price[out_box[j]] = res[j].price;
      se[out_box[j]] = res[j].std_err;
    }
  }
  for (int64_t i = 0; i < n; ++i) price_out[i] = price[i];
  if (std_err_out)
    for (int64_t i = 0; i < n; ++i) std_err_out[i] = se[i];
  if (route_out) {
    for (int64_t i : in_box) route_out[i] = 0;
    for (int64_t i : out_box) route_out[i] = 1;
  }
  return PMC_OK;
}

// File layout (native byte order): the 8 bytes "PMCMLP2\n", int32 n_in,
// int32 width, float64 y_scale, float64 lo[n_in], float64 hi[n_in],
// int64 n_params, float32 master weights [n_params] (W1 b1 .. W4 b4).
// Format 2 is the network with the tanh form of GELU; format 1 files (the
// erf form) are refused, since their weights belong to another function.
static const char kMlpMagic[8] = {'P', 'M', 'C', 'M', 'L', 'P', '2', '\n'};

extern "C" int pmc_mlp_save(const pmc_mlp* m, const char* path) {
  if (!m || !path) return PMC_E_ARG;
  std::vector<float> w((size_t)m->n_params);
  int rc = pmc_mlp_get_params(m, w.data());
  if (rc != PMC_OK) return rc;
  pmc_mlp* M = const_cast<pmc_mlp*>(m);
  FILE* f = std::fopen(path, "wb");
  if (!f) return ctx_fail(M->ctx, PMC_E_ARG, std::string("cannot open ") + path + " for writing");
  const int32_t n_in = m->n_in, width = m->width;
  const int64_t np = m->n_params;
  bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(&n_in, 4, 1, f) == 1 &&
            std::fwrite(&width, 4, 1, f) == 1 && std::fwrite(&m->y_scale, 8, 1, f) == 1 &&
            std::fwrite(m->lo.data(), 8, n_in, f) == (size_t)n_in &&
            std::fwrite(m->hi.data(), 8, n_in, f) == (size_t)n_in && std::fwrite(&np, 8, 1, f) == 1 &&
            std::fwrite(w.data(), 4, w.size(), f) == w.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return ctx_fail(M->ctx, PMC_E_ARG, std::string("write failed: ") + path);
  return PMC_OK;
}

extern "C" int pmc_mlp_load(pmc_ctx* ctx, const char* path, pmc_mlp** out) {
  if (!ctx || !path || !out) return PMC_E_ARG;
  FILE* f = std::fopen(path, "rb");
  if (!f) return ctx_fail(ctx, PMC_E_ARG, std::string("cannot open ") + path);
  char magic[8];
  int32_t n_in = 0, width = 0;
  double y_scale = 0;
  int64_t np = -1;
  std::vector<double> lo, hi;
  std::vector<float> w;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
            std::fread(&n_in, 4, 1, f) == 1 && std::fread(&width, 4, 1, f) == 1 &&
            std::fread(&y_scale, 8, 1, f) == 1 && n_in >= 1 && n_in <= 16 && width >= 32 && width <= 1024;
  if (ok) {
    lo.resize(n_in);
    hi.resize(n_in);
    ok = std::fread(lo.data(), 8, n_in, f) == (size_t)n_in && std::fread(hi.data(), 8, n_in, f) == (size_t)n_in &&
         std::fread(&np, 8, 1, f) == 1;
  }
  const int64_t want = (int64_t)width * n_in + width + 2 * ((int64_t)width * width + width) + width + 1;
  if (ok) ok = np == want;
  if (ok) {
    w.resize((size_t)np);
    ok = std::fread(w.data(), 4, w.size(), f) == w.size();
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;   // nothing after the weights
  }
  std::fclose(f);
  if (!ok) return ctx_fail(ctx, PMC_E_PARSE, std::string("not a surrogate file of this library: ") + path);
  pmc_mlp* m = nullptr;
  int rc = pmc_mlp_create(ctx, n_in, width, 0, lo.data(), hi.data(), y_scale, &m);
  if (rc != PMC_OK) return rc;
  rc = pmc_mlp_set_params(m, w.data());
  if (rc != PMC_OK) { pmc_mlp_free(m); return rc; }
  *out = m;
  return PMC_OK;
}
