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

#include "kernels.h"

namespace pmc {
namespace {

// ------------------------------------------------------------ Philox ------
// Philox4x32-10 (Salmon et al., SC'11): two 32x32 multiplications per round,
// swap-and-xor with the key, Weyl key bump between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// ---------------------------------------------- uniforms and normals -----
template <typename T> struct Num;

// FP32: u = (x>>9 + 1/2) 2^-23 (exact in binary32); Phi^-1 by AS241's
// 7-digit variant PPND7 (Wichura 1988).
template <> struct Num<float> {
  static __device__ __forceinline__ float uniform(uint32_t x) {
    return fmaf((float)(x >> 9), 0x1p-23f, 0x1p-24f);
  }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float normal(float p) {
    const float q = p - 0.5f;
    // central region |q| <= 0.425
    const float r = 0.180625f - q * q;
    const float nc = q * fmaf(fmaf(fmaf(59.109374720f, r, 159.29113202f), r, 50.434271938f), r, 3.3871327179f);
    const float dc = fmaf(fmaf(fmaf(67.187563600f, r, 78.757757664f), r, 17.895169469f), r, 1.0f);
    // tails: r = sqrt(-log(min(p, 1-p))); 1-p is exact for our uniforms
    const float pt = fminf(p, 1.0f - p);
    const float rt = __builtin_sqrtf(-__logf(pt));
    float s = rt - 1.6f;
    float nt = fmaf(fmaf(fmaf(0.17023821103f, s, 1.3067284816f), s, 2.7568153900f), s, 1.4234372777f);
    float dt = fmaf(fmaf(0.12021132975f, s, 0.73700164250f), s, 1.0f);
    const bool far = rt > 5.0f;
    if (__any(far)) {   // min(p,1-p) < e^-25: unreachable for 23-bit uniforms, kept for completeness
      const float e = rt - 5.0f;
      const float ne = fmaf(fmaf(fmaf(0.017337203997f, e, 0.42868294337f), e, 3.0812263860f), e, 6.6579051150f);
      const float de = fmaf(fmaf(0.012258202635f, e, 0.24197894225f), e, 1.0f);
      nt = far ? ne : nt;
      dt = far ? de : dt;
    }
    const bool central = fabsf(q) <= 0.425f;
    const float num = central ? nc : copysignf(nt, q);
    const float den = central ? dc : dt;
    return num * rcp(den);
  }
  static __device__ __forceinline__ float expv(float x) { return __expf(x); }
  static __device__ __forceinline__ float div(float a, float b) { return a * rcp(b); }
};

// FP64: u = (x + 1/2) 2^-32 (exact); Phi^-1 by AS241 PPND16.
template <> struct Num<double> {
  static __device__ __forceinline__ double uniform(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }
  static __device__ double normal(double p) {
    const double q = p - 0.5;
    if (fabs(q) <= 0.425) {
      const double r = 0.180625 - q * q;
      const double n = ((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r +
                             6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r +
                           1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r +
                         1.3314166789178437745e+2) * r + 3.3871328727963666080e0;
      const double d = ((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r +
                             3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r +
                           5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r +
                         4.2313330701600911252e+1) * r + 1.0;
      return q * n / d;
    }
    double r = q < 0 ? p : 1.0 - p;
    r = sqrt(-log(r));
    double v;
    if (r <= 5.0) {
      r -= 1.6;
      const double n = ((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r +
                             2.41780725177450611770e-1) * r + 1.27045825245236838258e0) * r +
                           3.64784832476320460504e0) * r + 5.76949722146069140550e0) * r +
                         4.63033784615654529590e0) * r + 1.42343711074968357734e0;
      const double d = ((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r +
                             1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r +
                           6.89767334985100004550e-1) * r + 1.67638483018380384940e0) * r +
                         2.05319162663775882187e0) * r + 1.0;
      v = n / d;
    } else {
      r -= 5.0;
      const double n = ((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
                             1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r +
                           2.96560571828504891230e-1) * r + 1.78482653991729133580e0) * r +
                         5.46378491116411436990e0) * r + 6.65790464350110377720e0;
      const double d = ((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r +
                             1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r +
                           1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
                         5.99832206555887937690e-1) * r + 1.0;
      v = n / d;
    }
    return q < 0 ? -v : v;
  }
  static __device__ __forceinline__ double expv(double x) { return exp(x); }
  static __device__ __forceinline__ double div(double a, double b) { return a / b; }
};

template <typename T>
struct Args {
  const Instr* code;
  const T* consts;
  const InstDesc* desc;
  const int32_t* itab;
  const T* rtab;
  const double* chol;
  const uint32_t* sobol;
  int sobol_bits;
  const int2* work;
  int n_work;
  uint32_t* queue;
  double2* partial;
  T* payoff_out;
  const T* paths;
  uint32_t k0, k1;
  int ppt;
  int n_assets;
};

template <typename T>
Args<T> typed(const McLaunch& a) {
  Args<T> g;
  g.code = a.code; g.consts = (const T*)a.consts; g.desc = a.desc; g.itab = a.itab;
  g.rtab = (const T*)a.rtab; g.chol = a.chol; g.sobol = a.sobol; g.sobol_bits = a.sobol_bits;
  g.work = a.work; g.n_work = a.n_work; g.queue = a.queue; g.partial = a.partial;
  g.payoff_out = (T*)a.payoff_out; g.paths = (const T*)a.paths; g.k0 = a.k0; g.k1 = a.k1;
  g.ppt = a.ppt; g.n_assets = a.n_assets;
  return g;
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// ------------------------------------------------------- path sources -----
// Per-instance model constants, uniform across the wave.
template <typename T, int A>
struct Model {
  T mu[A], sig[A], s0[A];
  T L[A][A];
  __device__ __forceinline__ void load(const Args<T>& g, const InstDesc& D) {
    const T* m = g.rtab + D.model_off;
#pragma unroll
    for (int a = 0; a < A; ++a) { mu[a] = m[a]; sig[a] = m[A + a]; s0[a] = m[2 * A + a]; }
    const double* l = g.chol + D.chol_off;
#pragma unroll
    for (int i = 0; i < A; ++i)
#pragma unroll
      for (int j = 0; j < A; ++j) L[i][j] = (T)l[i * A + j];
  }
};

// Generates the path of one lane slot by slot into the window.
template <typename T, int RNG, int A>
struct GenSource {
  static constexpr int WS = kWindow / A;   // slots held in the window
  T x[A];
  int base;        // first slot in the window (uniform), -1 if empty
  int next_slot;   // next slot to generate (uniform)
  uint32_t blk;    // Philox block held in buf (uniform)
  uint32_t buf[4];
  uint32_t path, gray;
  uint32_t k0, k1, inst;
  int n_slots, sobol_bits;
  const uint32_t* sobol;
  const T* slotc;
  const T* spotp;
  Model<T, A> M;

  __device__ __forceinline__ void init(const Args<T>& g, const InstDesc& d, uint32_t p) {
    path = p; gray = p ^ (p >> 1);
    k0 = g.k0; k1 = g.k1; inst = d.instance;
    n_slots = d.n_slots; sobol_bits = g.sobol_bits; sobol = g.sobol;
    M.load(g, d);
    slotc = g.rtab + d.slot_off;
    spotp = g.rtab + d.model_off + 2 * A;
    base = -1; next_slot = 0; blk = 0xFFFFFFFFu;
#pragma unroll
    for (int a = 0; a < A; ++a) x[a] = T(0);
  }

  __device__ __forceinline__ uint32_t word(uint32_t w) {
    if (RNG == 0) {
      const uint32_t b = w >> 2;
      if (b != blk) {
        philox4x32_10(path, b, inst, 0u, k0, k1, buf);
        blk = b;
      }
      const uint32_t j = w & 3u;
      return j == 0 ? buf[0] : j == 1 ? buf[1] : j == 2 ? buf[2] : buf[3];
    } else {
      const uint32_t* v = sobol + (size_t)w * 32u;
      uint32_t acc = 0;
      for (int b = 0; b < sobol_bits; ++b) acc ^= v[b] & (0u - ((gray >> b) & 1u));
      return acc;
    }
  }

  // one GBM step to slot q (all assets); optionally record words/normals
  __device__ __forceinline__ void step(int q, uint32_t* wout, T* zout, uint32_t npath) {
    T z[A];
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const uint32_t w = (uint32_t)(q * A + a);
      const uint32_t x32 = word(w);
      z[a] = Num<T>::normal(Num<T>::uniform(x32));
      if (wout) wout[(size_t)w * npath + path] = x32;
      if (zout) zout[(size_t)w * npath + path] = z[a];
    }
    const T dt = slotc[2 * q], sdt = slotc[2 * q + 1];
#pragma unroll
    for (int a = 0; a < A; ++a) {
      T wa = T(0);
#pragma unroll
      for (int k = 0; k <= a; ++k) wa += M.L[a][k] * z[k];
      x[a] = x[a] + M.mu[a] * dt + (M.sig[a] * sdt) * wa;
    }
  }

  __device__ __forceinline__ void refill(T (&win)[kWindow], int s) {
    if (s < next_slot) {            // backward read: regenerate from the spot
#pragma unroll
      for (int a = 0; a < A; ++a) x[a] = T(0);
      next_slot = 0;
    }
    while (next_slot < s) { step(next_slot, nullptr, nullptr, 0); ++next_slot; }
    const int cnt = min(WS, n_slots - s);
#pragma unroll
    for (int j = 0; j < WS; ++j) {
      if (j < cnt) {
        step(s + j, nullptr, nullptr, 0);
#pragma unroll
        for (int a = 0; a < A; ++a) win[j * A + a] = M.s0[a] * Num<T>::expv(x[a]);
      }
    }
    next_slot = s + cnt;
    base = s;
  }

  __device__ __forceinline__ T read(T (&win)[kWindow], int slot, int a) {
    if (slot < base || slot >= base + WS || base < 0) refill(win, slot);
    const int i = uni((slot - base) * A + a) & (kWindow - 1);
    return win[i];
  }
  __device__ __forceinline__ T spot(int a) const { return spotp[a]; }
};

// Reads stored prices [slot][asset][path] through the same window.
template <typename T, int A>
struct MemSource {
  static constexpr int WS = kWindow / A;
  int base, n_slots;
  uint32_t path, n_paths;
  const T* paths;
  const T* spotp;

  __device__ __forceinline__ void init(const Args<T>& g, const InstDesc& d, uint32_t p) {
    path = p; n_paths = d.n_paths; n_slots = d.n_slots; base = -1;
    paths = g.paths;
    spotp = g.rtab + d.model_off + 2 * A;
  }
  __device__ __forceinline__ void refill(T (&win)[kWindow], int s) {
    const int last = n_slots - 1;
#pragma unroll
    for (int j = 0; j < WS; ++j) {
      const int q = min(s + j, last);
#pragma unroll
      for (int a = 0; a < A; ++a)
        win[j * A + a] = paths[((size_t)q * A + a) * n_paths + path];
    }
    base = s;
  }
  __device__ __forceinline__ T read(T (&win)[kWindow], int slot, int a) {
    if (slot < base || slot >= base + WS || base < 0) refill(win, slot);
    const int i = uni((slot - base) * A + a) & (kWindow - 1);
    return win[i];
  }
  __device__ __forceinline__ T spot(int a) const { return spotp[a]; }
};

// ------------------------------------------------------- interpreter ------
template <typename T, class Src>
__device__ __forceinline__ T interpret(const Args<T>& g, const InstDesc& D, Src& src, int* frames) {
  T R[kRegFile];
  T win[kWindow];
#pragma unroll
  for (int i = 0; i < kRegFile; ++i) R[i] = T(0);
#pragma unroll
  for (int i = 0; i < kWindow; ++i) win[i] = T(0);
  const int32_t* tt = g.itab + D.tt_off;
  const int32_t* dm = g.itab + D.daymap_off;
  int pc = 0, t0 = 0;
  int f_top = 0, f_rem = 0, f_t0 = 0, depth = 0;
  for (;;) {
    const uint2 w = *reinterpret_cast<const uint2*>(g.code + pc);
    const uint32_t w0 = (uint32_t)uni((int)w.x);
    const int imm = uni((int)w.y);
    const int op = w0 & 0xff, a = (w0 >> 16) & (kRegFile - 1), b = (w0 >> 24) & (kRegFile - 1);
    const int d = (w0 >> 8) & (kRegFile - 1);
    const int ai = (w0 >> 16) & 0xff;  // asset / party-pair operand
    ++pc;
    if (op == OP_HALT) break;
    const T ra = R[a], rb = R[b];
    T v = T(0);
    switch (op) {
      case OP_CONST: v = g.consts[imm]; break;
      case OP_PARAM: v = g.rtab[D.param_off + imm]; break;
      case OP_MODEL: {
        const int day = tt[imm] + t0;
        if (day <= 0) {
          v = src.spot(ai);
        } else {
          const int s = uni(dm[min(day, D.horizon)]);
          v = s < 0 ? src.spot(ai) : src.read(win, s, ai);
        }
        break;
      }
      case OP_TEXPR: v = (T)(tt[imm] + t0); break;
      case OP_NOW: v = (T)D.t_now; break;
      case OP_PAYOFF: {
        const int day = min(max(tt[imm] + t0, 0), D.horizon);
        v = (T)g.itab[D.sign_off + ai] * g.rtab[D.disc_off + day];
        break;
      }
      case OP_ADD: v = ra + rb; break;
      case OP_SUB: v = ra - rb; break;
      case OP_MUL: v = ra * rb; break;
      case OP_DIV: v = Num<T>::div(ra, rb); break;
      case OP_MIN: v = fmin(ra, rb); break;
      case OP_MAX: v = fmax(ra, rb); break;
      case OP_LT: v = ra < rb ? T(1) : T(0); break;
      case OP_LE: v = ra <= rb ? T(1) : T(0); break;
      case OP_EQ: v = ra == rb ? T(1) : T(0); break;
      case OP_AND: v = (ra != T(0) && rb != T(0)) ? T(1) : T(0); break;
      case OP_OR: v = (ra != T(0) || rb != T(0)) ? T(1) : T(0); break;
      case OP_NEG: v = -ra; break;
      case OP_NOT: v = ra == T(0) ? T(1) : T(0); break;
      case OP_SEL: v = ra != T(0) ? rb : R[imm & (kRegFile - 1)]; break;
      case OP_JNONE:
        if (!__any(ra != T(0))) pc = imm;
        break;
      case OP_JALL:
        if (__all(ra != T(0))) pc = imm;
        break;
      case OP_LOOP:
        if (depth > 0) {
          frames[3 * depth - 3] = f_top; frames[3 * depth - 2] = f_rem; frames[3 * depth - 1] = f_t0;
        }
        ++depth;
        f_top = pc; f_rem = tt[imm]; f_t0 = t0;
        break;
      case OP_LTAKE: {
        const bool take = ra == T(0) && R[d] != T(0);
        v = take ? T(1) : T(0);
        if (!__any(take)) pc = imm;
        break;
      }
      case OP_LMERGE: v = ra != T(0) ? rb : R[d]; break;
      case OP_LDONE: v = (R[d] != T(0) || ra != T(0)) ? T(1) : T(0); break;
      case OP_LNEXT:
        if (__all(ra != T(0))) {
          pc = imm;
        } else if (f_rem > 0) {
          --f_rem; ++t0; pc = f_top;
        }
        break;
      case OP_LELSE: v = ra != T(0) ? R[d] : rb; break;
      case OP_LEND:
        t0 = f_t0;
        --depth;
        if (depth > 0) {
          f_top = uni(frames[3 * depth - 3]); f_rem = uni(frames[3 * depth - 2]); f_t0 = uni(frames[3 * depth - 1]);
        }
        break;
      default: break;
    }
    R[d] = v;
  }
  return R[0];
}

// ------------------------------------------------------ reductions --------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Block sums of (s, ss); thread 0 gets the result.  red: 2 * (blockDim/64)
__device__ __forceinline__ void block_sum2(double& s, double& ss, double* red) {
  s = wave_sum(s);
  ss = wave_sum(ss);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) { red[2 * wv] = s; red[2 * wv + 1] = ss; }
  __syncthreads();
  if (threadIdx.x == 0) {
    s = 0; ss = 0;
    for (int i = 0; i < nw; ++i) { s += red[2 * i]; ss += red[2 * i + 1]; }
  }
  __syncthreads();
}

// ----------------------------------------------------------- kernels ------
// Work items are (instance, tile); a tile is ppt * blockDim paths of one
// instance.  Non-persistent launches take item = blockIdx.x of instance 0;
// persistent launches pull items from an atomic counter until none is left.
template <typename T, int RNG, int A, bool MEM>
__global__ __launch_bounds__(256) void k_mc(Args<T> g) {
  __shared__ double red[8];
  __shared__ int frames_all[4][3 * kMaxLoopDepth];
  __shared__ int item_s;
  int* frames = frames_all[threadIdx.x >> 6];
  int item = blockIdx.x;
  for (;;) {
    if (g.queue) {
      if (threadIdx.x == 0) item_s = (int)atomicAdd(g.queue, 1u);
      __syncthreads();
      item = item_s;
      __syncthreads();
    }
    if (item >= g.n_work) break;
    const int2 wi = g.work ? g.work[item] : make_int2(0, item);
    const InstDesc& D = g.desc[wi.x];
    double s = 0.0, ss = 0.0;
    for (int r = 0; r < g.ppt; ++r) {
      const uint32_t path = ((uint32_t)wi.y * (uint32_t)g.ppt + (uint32_t)r) * blockDim.x + threadIdx.x;
      const bool valid = path < D.n_paths;
      const uint32_t p = valid ? path : D.n_paths - 1;
      T v;
      if (MEM) {
        MemSource<T, A> src;
        src.init(g, D, p);
        v = interpret<T>(g, D, src, frames);
      } else {
        GenSource<T, RNG, A> src;
        src.init(g, D, p);
        v = interpret<T>(g, D, src, frames);
      }
      if (valid) {
        const double x = (double)v;
        s += x; ss += x * x;
        if (g.payoff_out) g.payoff_out[path] = v;
      }
    }
    block_sum2(s, ss, red);
    if (threadIdx.x == 0) g.partial[D.first_item + wi.y] = make_double2(s, ss);
    if (!g.queue) break;
  }
}

// Two-phase path generation: stored prices [slot][asset][path].
template <typename T, int RNG, int A>
__global__ __launch_bounds__(256) void k_pathgen(Args<T> g, T* out, uint32_t* wout, T* zout, uint32_t n_paths) {
  const uint32_t path = blockIdx.x * blockDim.x + threadIdx.x;
  if (path >= n_paths) return;
  const InstDesc& D = g.desc[0];
  GenSource<T, RNG, A> src;
  src.init(g, D, path);
  for (int q = 0; q < D.n_slots; ++q) {
    src.step(q, wout, zout, n_paths);
#pragma unroll
    for (int a = 0; a < A; ++a)
      out[((size_t)q * A + a) * n_paths + path] = src.M.s0[a] * Num<T>::expv(src.x[a]);
  }
}

// Deterministic per-instance sum of the work-item partials: one block per
// instance, fixed summation order.
__global__ __launch_bounds__(256) void k_reduce(const double2* partial, const InstDesc* desc, double2* out) {
  __shared__ double red[8];
  const InstDesc& D = desc[blockIdx.x];
  double s = 0.0, ss = 0.0;
  for (uint32_t i = threadIdx.x; i < D.n_tiles; i += blockDim.x) {
    const double2 p = partial[D.first_item + i];
    s += p.x; ss += p.y;
  }
  block_sum2(s, ss, red);
  if (threadIdx.x == 0) out[blockIdx.x] = make_double2(s, ss);
}

// FP64 Cholesky-Banachiewicz, one matrix per thread (m <= 4 in practice).
__global__ void k_cholesky(const double* a, double* l, int* bad, int n, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* A_ = a + (size_t)i * m * m;
  double* L = l + (size_t)i * m * m;
  int ok = 1;
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) L[r * m + c] = 0.0;
  for (int r = 0; r < m && ok; ++r) {
    for (int c = 0; c <= r; ++c) {
      double s = A_[r * m + c];
      for (int k = 0; k < c; ++k) s -= L[r * m + k] * L[c * m + k];
      if (r == c) {
        if (!(s > 0.0)) { ok = 0; break; }
        L[r * m + r] = sqrt(s);
      } else {
        L[r * m + c] = s / L[c * m + c];
      }
    }
  }
  if (!ok) atomicMin(bad, i);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T, int RNG, int A>
hipError_t mc_launch_t(bool mem, const McLaunch& a, int grid, int block, hipStream_t s) {
  Args<T> g = typed<T>(a);
  if (mem) hipLaunchKernelGGL((k_mc<T, RNG, A, true>), dim3(grid), dim3(block), 0, s, g);
  else hipLaunchKernelGGL((k_mc<T, RNG, A, false>), dim3(grid), dim3(block), 0, s, g);
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
int occ_t(int block) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mc<T, RNG, A, false>, block, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace

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

hipError_t launch_reduce(const double2* partial, const InstDesc* desc, int n_inst, double2* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(n_inst), dim3(256), 0, s, partial, desc, out);
  return hipGetLastError();
}

hipError_t launch_cholesky(const double* a, double* l, int* bad, int n, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_cholesky, dim3((n + 255) / 256), dim3(256), 0, s, a, l, bad, n, m);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

int mc_occupancy(int precision, int rng, int n_assets, int block) {
#define OCC(T, R) \
  switch (n_assets) { case 1: return occ_t<T, R, 1>(block); case 2: return occ_t<T, R, 2>(block); \
                      case 3: return occ_t<T, R, 3>(block); default: return occ_t<T, R, 4>(block); }
  if (precision == 1) { if (rng) { OCC(double, 1) } else { OCC(double, 0) } }
  if (rng) { OCC(float, 1) } else { OCC(float, 0) }
#undef OCC
}

}  // namespace pmc
