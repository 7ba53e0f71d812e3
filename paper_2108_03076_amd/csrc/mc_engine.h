// Device engine of the Monte Carlo pricer: random streams, normals, path
// sources, the bytecode interpreter, reductions and the kernel body that
// drives them.  Included by the static kernels (mc_kernels.hip) and, as text,
// by the payoff code generator, whose run-time compiled kernels reuse this
// body with a generated payoff function in place of the interpreter.
#pragma once
#include "pmc_device.h"

namespace pmc {
namespace eng {

// ------------------------------------------------------------ Philox ------
// Philox4x32-10 (Salmon et al., SC'11): two 32x32 multiplications per round,
// swap-and-xor with the key, Weyl key bump between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 product each (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u, p1 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
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

// FP32: u = (x>>9 + 1/2) 2^-23 (exact in binary32, 2^-24 <= u <= 1 - 2^-24).
// Phi^-1 through the change of variable of Giles ("Approximating the erfinv
// function", 2011): w = -ln(4u(1-u)), z = (2u-1) g(w), with g a polynomial in
// w - 2.5 for w < 5 and in sqrt(w) - c for the tail (w <= 15.25 for these
// uniforms).  Our own coefficients, fitted by paper_2108_03076_amd/fit_normal.py;
// |z - Phi^-1(u)| <= 3e-7 max(1, |z|) over the binary32 uniforms.
template <> struct Num<float> {
  static __device__ __forceinline__ float uniform(uint32_t x) {
    return fmaf((float)(x >> 9), 0x1p-23f, 0x1p-24f);
  }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  // f = 1 + (x >> 9) 2^-23; u = f - (1 - 2^-24) is exact (Sterbenz), and
  // 1 - u and 2u - 1 = u - (1 - u) are multiples of 2^-24 below 1: exact.
  static __device__ __forceinline__ float word_u(uint32_t x) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9u)) - 0x1.fffffep-1f;
  }
  static __device__ __forceinline__ float normal_word(uint32_t x) {
    const float u = word_u(x);
    return (u - (1.0f - u)) * normal_g(u);
  }
  // s Phi^-1(u) with the scale taken into 2u - 1: one rounding of (2u - 1) s
  // (2s is exact), then the same g(w).
  static __device__ __forceinline__ float normal_word_scaled(uint32_t x, float s) {
    const float u = word_u(x);
    return fmaf(u, 2.0f * s, -s) * normal_g(u);
  }
  // Log-prices are held in units of log2 (a price is s0 2^x): one
  // exponential instruction per price.
  static constexpr float kLog = 1.4426950408889634f;
  static __device__ __forceinline__ float exps(float x) { return __builtin_amdgcn_exp2f(x); }
  static __device__ __forceinline__ float normal_g(float u) {
    // t = u (1 - u) rounded once: 1 - u is exact, so this is the same value
    // as the product u * (1 - u), in one instruction
    const float t = fmaf(-u, u, u);
    // d = w - 2.5 = -ln2 (log2 t + 2) - 2.5
    const float d = fmaf(__builtin_amdgcn_logf(t), -0x1.62e430p-1f, -0x1.f17218p+1f);
    float g = 3.9583209598959e-08f;
    g = fmaf(g, d, 4.851791004512052e-07f);
    g = fmaf(g, d, -4.981194706488168e-06f);
    g = fmaf(g, d, -6.207880232977914e-06f);
    g = fmaf(g, d, 0.00030911510111764073f);
    g = fmaf(g, d, -0.001773041789419949f);
    g = fmaf(g, d, -0.00590812973678112f);
    g = fmaf(g, d, 0.34880268573760986f);
    g = fmaf(g, d, 2.1233136653900146f);
    const bool tail = d >= 2.5f;   // w >= 5: 0.34% of draws
    if (__builtin_expect(__any(tail), 0)) {
      const float e = __builtin_amdgcn_sqrtf(d + 2.5f) - 3.071047627109653f;
      float h = -0.0003539455065038055f;
      h = fmaf(h, e, -4.474368324736133e-05f);
      h = fmaf(h, e, 0.0020311614498496056f);
      h = fmaf(h, e, -0.004341235384345055f);
      h = fmaf(h, e, 0.006380986422300339f);
      h = fmaf(h, e, -0.008731475099921227f);
      h = fmaf(h, e, 0.011283238418400288f);
      h = fmaf(h, e, 1.4183263778686523f);
      h = fmaf(h, e, 4.107142925262451f);
      g = tail ? h : g;
    }
    return g;
  }
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
  static __device__ __forceinline__ double normal_word(uint32_t x) { return normal(uniform(x)); }
  static __device__ __forceinline__ double normal_word_scaled(uint32_t x, double s) { return s * normal_word(x); }
  // natural log-prices (a price is s0 e^x)
  static constexpr double kLog = 1.0;
  static __device__ __forceinline__ double exps(double x) { return exp(x); }
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
  const uint32_t* sobol_hi;   // [path / 64][dim]: Sobol bits 6.. of each wave's points, or null
  int sobol_dims;
  const int* order;      // instances in processing order (longest first), or null
  int tiles;             // work items (path tiles) per instance
  int n_work;
  uint32_t* queue;
  double2* partial;
  uint32_t* done;        // batches: per-instance finished tiles (zero at launch)
  double2* result;       // per instance: (sum, sum of squares); batches: written by the block that
                         // finishes the instance's last tile (one instrument: by k_finish)
  const double* chol_in; // correlation matrices (A x A per instance)
  int* status;           // per instance: 0, or 1 if the correlation is not positive definite
  int factor;            // 1: each block factors instance 0's matrix itself (single instrument)
  T* payoff_out;
  const T* paths;
  uint32_t k0, k1;
  int ppt;
  int n_assets;
};


__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Read-only tables (bytecode, descriptors, time tables, discount factors,
// model constants, direction numbers) are read through the constant address
// space so that uniform reads become scalar loads through the scalar cache.
template <typename T>
using kptr = const __attribute__((address_space(4))) T*;
template <typename T>
using lptr = const __attribute__((address_space(3))) T*;
template <typename T>
using lwptr = __attribute__((address_space(3))) T*;
template <typename T>
__device__ __forceinline__ kptr<T> K(const T* p) { return (kptr<T>)p; }

__device__ __forceinline__ InstDesc load_desc(const InstDesc* base, int i) {
  InstDesc d;
  kptr<int32_t> src = K(reinterpret_cast<const int32_t*>(base + i));
  int32_t* dst = reinterpret_cast<int32_t*>(&d);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(InstDesc) / 4); ++k) dst[k] = src[k];
  return d;
}

// ------------------------------------------------------- path sources -----
// A wave-uniform value, marked as such (kept in scalar registers).
__device__ __forceinline__ float uniform_value(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform_value(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll)), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Per-instance model constants, uniform across the wave.
template <typename T, int A>
struct Model {
  // Per unit time and in the log units of Num<T>: drift dr = kLog (r - sigma^2/2)
  // and diffusion C = kLog sigma_a L_ak, so a step is
  // x_a += dr_a dt + sum_k C_ak (sqrt(dt) z_k).
  T dr[A], s0[A];
  T C[A][A];
  // The diffusion factor comes from the prepared FP64 Cholesky table, or
  // (own) from the block's own coefficients, already made (lf: C row-major,
  // then dr).
  __device__ __forceinline__ void load(const Args<T>& g, const InstDesc& D, const T* lf, bool own) {
    kptr<T> m = K(g.rtab) + D.model_off;
#pragma unroll
    for (int a = 0; a < A; ++a) s0[a] = m[2 * A + a];
    if (own) {
#pragma unroll
      for (int i = 0; i < A; ++i) {
        dr[i] = lf[A * A + i];
#pragma unroll
        for (int j = 0; j < A; ++j) C[i][j] = lf[i * A + j];
      }
    } else {
      kptr<double> l = K(g.chol) + D.chol_off;
#pragma unroll
      for (int i = 0; i < A; ++i) {
        dr[i] = drift_coef(m[i]);
#pragma unroll
        for (int j = 0; j < A; ++j) C[i][j] = diffusion_coef(l[i * A + j], m[A + i]);
      }
    }
  }
  // the same arithmetic wherever the coefficients are made, so that a path
  // is the same bit for bit whichever kernel generates it
  static __device__ __forceinline__ T drift_coef(T mu) { return mu * Num<T>::kLog; }
  static __device__ __forceinline__ T diffusion_coef(double l, T sig) { return ((T)l * sig) * Num<T>::kLog; }
};

// FP64 Cholesky-Banachiewicz (row by row) of the m x m matrix a into the
// lower triangle of l (upper part zeroed); false if a is not positive
// definite.  Used by the preparation kernel and by blocks that factor their
// instrument's matrix themselves, so both give the same factor bit for bit.
template <typename PA, typename PL>
__device__ __forceinline__ bool chol_factor(PA a, PL l, int m) {
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) l[r * m + c] = 0.0;
  for (int r = 0; r < m; ++r) {
    for (int c = 0; c <= r; ++c) {
      double s = a[r * m + c];
      for (int k = 0; k < c; ++k) s -= l[r * m + k] * l[c * m + k];
      if (r == c) {
        if (!(s > 0.0)) return false;
        l[r * m + r] = sqrt(s);
      } else {
        l[r * m + c] = s / l[c * m + c];
      }
    }
  }
  return true;
}

// ------------------------------------------------------ lane vectors -----
// The two-phase evaluator may give each lane P consecutive paths: the
// generated payoff then computes on P-wide values and decisions, while its
// wave-uniform work (loop shift and counters, day->slot lookups, window
// management) is shared by the P paths and the stored prices of a slot come
// in one P-wide load.  For P = 1 the types are plain T and bool and every
// helper below is the scalar operation itself, so a compiled payoff computes
// exactly what the interpreter computes.
template <typename T, int P>
struct alignas(sizeof(T) * P) LaneVec {
  T v[P];
  LaneVec() = default;
  __device__ __forceinline__ LaneVec(T x) {
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = x;
  }
};
// P decisions of one lane.  For P > 2, bits 0..P-1 of a vector register:
// their logic is one vector instruction for all P paths (as P separate
// booleans it became P 64-bit lane masks on the scalar unit, which bounds the
// stored-path evaluator).  For P <= 2, P booleans (wave-wide lane masks):
// each comparison and selection is then one vector instruction per path and
// the logic scalar, where packing and testing bits would cost several vector
// instructions per decision.
template <int P>
struct LaneMask {
  static constexpr bool kBools = P <= 2;
  static constexpr uint32_t kAll = (1u << P) - 1u;
  uint32_t m;      // P > 2
  bool b[P];       // P <= 2
  LaneMask() = default;
  __device__ __forceinline__ LaneMask(bool x) {
    if constexpr (kBools) {
#pragma unroll
      for (int i = 0; i < P; ++i) b[i] = x;
    } else {
      m = x ? kAll : 0u;
    }
  }
  __device__ __forceinline__ bool bit(int i) const {
    if constexpr (kBools) return b[i];
    else return (m >> i) & 1u;
  }
};
template <bool B, class X, class Y> struct pick_t { using type = X; };
template <class X, class Y> struct pick_t<false, X, Y> { using type = Y; };
template <typename T, int P>
using VecT = typename pick_t<P == 1, T, LaneVec<T, P>>::type;
template <int P>
using MaskT = typename pick_t<P == 1, bool, LaneMask<P>>::type;

template <typename T> __device__ __forceinline__ T lane_elem(T x, int) { return x; }
template <typename T, int P> __device__ __forceinline__ T lane_elem(const LaneVec<T, P>& x, int i) { return x.v[i]; }

#define PMC_VEC_BINARY(NAME, EXPR)                                                              \
  template <typename T>                                                                         \
  __device__ __forceinline__ T NAME(T a, T b) { return EXPR; }                                  \
  template <typename T, int P>                                                                  \
  __device__ __forceinline__ LaneVec<T, P> NAME(const LaneVec<T, P>& x, const LaneVec<T, P>& y) { \
    LaneVec<T, P> r;                                                                            \
    _Pragma("unroll") for (int i = 0; i < P; ++i) {                                             \
      const T a = x.v[i], b = y.v[i];                                                           \
      r.v[i] = EXPR;                                                                            \
    }                                                                                           \
    return r;                                                                                   \
  }
PMC_VEC_BINARY(vadd, a + b)
PMC_VEC_BINARY(vsub, a - b)
PMC_VEC_BINARY(vmul, a * b)
PMC_VEC_BINARY(vdiv, Num<T>::div(a, b))
PMC_VEC_BINARY(vmin, fmin(a, b))
PMC_VEC_BINARY(vmax, fmax(a, b))
#undef PMC_VEC_BINARY

#define PMC_VEC_COMPARE(NAME, OP)                                                                   \
  template <typename T>                                                                             \
  __device__ __forceinline__ bool NAME(T a, T b) { return a OP b; }                                 \
  template <typename T, int P>                                                                      \
  __device__ __forceinline__ LaneMask<P> NAME(const LaneVec<T, P>& x, const LaneVec<T, P>& y) {     \
    LaneMask<P> r;                                                                                  \
    if constexpr (LaneMask<P>::kBools) {                                                            \
      _Pragma("unroll") for (int i = 0; i < P; ++i) r.b[i] = x.v[i] OP y.v[i];                      \
    } else {                                                                                        \
      r.m = 0u;                                                                                     \
      _Pragma("unroll") for (int i = 0; i < P; ++i) r.m |= (x.v[i] OP y.v[i]) ? (1u << i) : 0u;     \
    }                                                                                               \
    return r;                                                                                       \
  }
PMC_VEC_COMPARE(vlt, <)
PMC_VEC_COMPARE(vle, <=)
PMC_VEC_COMPARE(veq, ==)
#undef PMC_VEC_COMPARE

template <typename T> __device__ __forceinline__ T vneg(T a) { return -a; }
template <typename T, int P> __device__ __forceinline__ LaneVec<T, P> vneg(const LaneVec<T, P>& x) {
  LaneVec<T, P> r;
#pragma unroll
  for (int i = 0; i < P; ++i) r.v[i] = -x.v[i];
  return r;
}
__device__ __forceinline__ bool vnot(bool a) { return !a; }
__device__ __forceinline__ bool vand(bool a, bool b) { return a && b; }
__device__ __forceinline__ bool vor(bool a, bool b) { return a || b; }
__device__ __forceinline__ bool vany(bool a) { return __any(a); }
__device__ __forceinline__ bool vall(bool a) { return __all(a); }
template <typename T> __device__ __forceinline__ T vsel(bool c, T a, T b) { return c ? a : b; }
template <int P> __device__ __forceinline__ LaneMask<P> vnot(const LaneMask<P>& a) {
  LaneMask<P> r;
  if constexpr (LaneMask<P>::kBools) {
#pragma unroll
    for (int i = 0; i < P; ++i) r.b[i] = !a.b[i];
  } else {
    r.m = a.m ^ LaneMask<P>::kAll;
  }
  return r;
}
template <int P> __device__ __forceinline__ LaneMask<P> vand(const LaneMask<P>& a, const LaneMask<P>& b) {
  LaneMask<P> r;
  if constexpr (LaneMask<P>::kBools) {
#pragma unroll
    for (int i = 0; i < P; ++i) r.b[i] = a.b[i] && b.b[i];
  } else {
    r.m = a.m & b.m;
  }
  return r;
}
template <int P> __device__ __forceinline__ LaneMask<P> vor(const LaneMask<P>& a, const LaneMask<P>& b) {
  LaneMask<P> r;
  if constexpr (LaneMask<P>::kBools) {
#pragma unroll
    for (int i = 0; i < P; ++i) r.b[i] = a.b[i] || b.b[i];
  } else {
    r.m = a.m | b.m;
  }
  return r;
}
template <int P> __device__ __forceinline__ bool vany(const LaneMask<P>& a) {
  if constexpr (LaneMask<P>::kBools) {
    bool x = false;
#pragma unroll
    for (int i = 0; i < P; ++i) x = x || a.b[i];
    return __any(x);
  } else {
    return __any(a.m != 0u);
  }
}
template <int P> __device__ __forceinline__ bool vall(const LaneMask<P>& a) {
  if constexpr (LaneMask<P>::kBools) {
    bool x = true;
#pragma unroll
    for (int i = 0; i < P; ++i) x = x && a.b[i];
    return __all(x);
  } else {
    return __all(a.m == LaneMask<P>::kAll);
  }
}
template <typename T, int P>
__device__ __forceinline__ LaneVec<T, P> vsel(const LaneMask<P>& c, const LaneVec<T, P>& a, const LaneVec<T, P>& b) {
  LaneVec<T, P> r;
#pragma unroll
  for (int i = 0; i < P; ++i) r.v[i] = c.bit(i) ? a.v[i] : b.v[i];
  return r;
}
template <int P>
__device__ __forceinline__ LaneMask<P> vsel(const LaneMask<P>& c, const LaneMask<P>& a, const LaneMask<P>& b) {
  LaneMask<P> r;
  if constexpr (LaneMask<P>::kBools) {
#pragma unroll
    for (int i = 0; i < P; ++i) r.b[i] = c.b[i] ? a.b[i] : b.b[i];
  } else {
    r.m = (c.m & a.m) | (~c.m & b.m & LaneMask<P>::kAll);
  }
  return r;
}

// Window bookkeeping of the sliding path sources: base is the window's first
// slot, kNoWindow while it is empty; a slot outside [base, base + ws) takes
// one unsigned comparison (slots are below 2^30).
constexpr int kNoWindow = -(1 << 30);
__device__ __forceinline__ bool outside(int slot, int base, int ws) {
  return (uint32_t)(slot - base) >= (uint32_t)ws;
}

// Price of asset a on a history day: entry day - first of its row of the
// history table, clamped to the row (flat before the first day).
template <typename T>
__device__ __forceinline__ T hist_value(kptr<T> h, int first, int n, int a, int day) {
  return h[a * n + min(max(day - first, 0), n - 1)];
}

// Generates the path of one lane slot by slot into the window.  CAP = 0:
// a window of kWindow values that slides forward and is regenerated from the
// spot on a backward read (paths of any length).  CAP > 0 (a power of two,
// at least n_slots * A): the whole path, generated once by prime() before
// the payoff runs; reads are register selects at a uniform index, and the
// generation code exists once in the kernel instead of at every read.
template <typename T, int RNG, int A, int CAP = 0>
struct GenSource {
  static_assert(CAP == 0 || (CAP & (CAP - 1)) == 0, "CAP is a power of two");
  using V = T;
  using Mask = bool;
  static constexpr int kWin = CAP > 0 ? CAP : kWindow;
  using Win = T[kWin];
  static constexpr int WS = kWindow / A;   // slots held in the sliding window
  T x[A];
  int base;        // first slot in the window (uniform), -1 if empty
  int next_slot;   // next slot to generate (uniform)
  uint32_t blk;    // Philox block held in buf0..buf3 (uniform)
  uint32_t buf0, buf1, buf2, buf3;
  uint32_t path, gray;
  uint32_t k0, k1, inst;
  int n_slots, sobol_bits, sobol_dims;
  kptr<uint32_t> sobol;
  kptr<uint32_t> sobol_hi;   // this wave's row of the high-part table
  lptr<uint32_t> lo;         // LDS table of low-bit XORs, at this lane's Gray bits
  bool use_lo;
  kptr<T> slotc;
  kptr<T> histp;
  int hist_first, n_hist;
  Model<T, A> M;

  __device__ __forceinline__ void init(const Args<T>& g, const InstDesc& d, uint32_t p, lptr<uint32_t> lo_tab,
                                       bool has_lo, const T* l_own = nullptr, bool own = false) {
    path = p; gray = p ^ (p >> 1);
    use_lo = RNG == 1 && has_lo;
    lo = lo_tab + (gray & 63u);
    k0 = g.k0; k1 = g.k1; inst = d.instance;
    n_slots = d.n_slots; sobol_bits = g.sobol_bits; sobol = K(g.sobol);
    sobol_dims = g.sobol_dims;
    sobol_hi = nullptr;
    if (RNG == 1 && g.sobol_hi) {
      // Points 64h .. 64h+63 of one wave share Gray-code bits 6 and up
      // (gray(p) >> 6 = gray(p >> 6)); their XOR of direction numbers is a
      // per-wave table entry, and only bits 0..5 remain per lane.
      const uint32_t h = (uint32_t)uni((int)(p >> 6));
      sobol_hi = K(g.sobol_hi) + (size_t)h * (size_t)sobol_dims;
    }
    M.load(g, d, l_own, own);
    slotc = K(g.rtab) + d.slot_off;
    histp = K(g.rtab) + d.hist_off;
    hist_first = d.hist_first; n_hist = d.n_hist;
    base = kNoWindow; next_slot = 0; blk = 0xFFFFFFFFu;
#pragma unroll
    for (int a = 0; a < A; ++a) x[a] = T(0);
  }

  __device__ __forceinline__ uint32_t word(uint32_t w) {
    if (RNG == 0) {
      const uint32_t b = w >> 2;
      if (b != blk) {
        uint32_t o[4];
        philox4x32_10(path, b, inst, 0u, k0, k1, o);
        buf0 = o[0]; buf1 = o[1]; buf2 = o[2]; buf3 = o[3];
        blk = b;
      }
      // four named registers and a select (an indexed array would be
      // demoted to scratch memory)
      const uint32_t j = w & 3u;
      const uint32_t lo2 = (j & 1u) ? buf1 : buf0;
      const uint32_t hi2 = (j & 1u) ? buf3 : buf2;
      return (j & 2u) ? hi2 : lo2;
    } else {
      kptr<uint32_t> v = sobol + (size_t)w * 32u;
      if (sobol_hi) {
        uint32_t acc = sobol_hi[w];
#pragma unroll
        for (int b = 0; b < 6; ++b) acc ^= v[b] & (0u - ((gray >> b) & 1u));
        return acc;
      }
      uint32_t acc = 0;
      for (int b = 0; b < sobol_bits; ++b) acc ^= v[b] & (0u - ((gray >> b) & 1u));
      return acc;
    }
  }

  // the A words of slot q (words q*A .. q*A+A-1); with the Sobol LDS table
  // the A loads are issued together (LO: the table is known to be there)
  template <bool LO = false>
  __device__ __forceinline__ void words(int q, uint32_t (&xw)[A]) {
    const uint32_t w0 = (uint32_t)(q * A);
    if (RNG == 1 && (LO || use_lo)) {
#pragma unroll
      for (int a = 0; a < A; ++a) xw[a] = sobol_hi[w0 + a] ^ lo[(w0 + a) * 64u];
    } else {
#pragma unroll
      for (int a = 0; a < A; ++a) xw[a] = word(w0 + a);
    }
  }

  // one GBM step from the slot's words and step sizes (dt, sqrt dt): the
  // normals come out scaled by sqrt dt, and each log-price takes its drift
  // and then its correlated terms (every addition on the log-price itself)
  __device__ __forceinline__ void advance(const uint32_t (&xw)[A], T dt, T sdt) {
    T zs[A];
#pragma unroll
    for (int a = 0; a < A; ++a) zs[a] = Num<T>::normal_word_scaled(xw[a], sdt);
#pragma unroll
    for (int a = 0; a < A; ++a) {
      T xa = x[a] + M.dr[a] * dt;
#pragma unroll
      for (int k = 0; k <= a; ++k) xa = xa + M.C[a][k] * zs[k];
      x[a] = xa;
    }
  }
  __device__ __forceinline__ T price(int a) const { return M.s0[a] * Num<T>::exps(x[a]); }

  // one GBM step to slot q (all assets); optionally record words/normals
  template <bool LO = false>
  __device__ __forceinline__ void step(int q, uint32_t* wout, T* zout, uint32_t npath) {
    uint32_t xw[A];
    words<LO>(q, xw);
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const size_t w = (size_t)(q * A + a);
      if (wout) wout[w * npath + path] = xw[a];
      if (zout) zout[w * npath + path] = Num<T>::normal_word(xw[a]);
    }
    advance(xw, slotc[2 * q], slotc[2 * q + 1]);
  }

  // Every slot of the path, in order, into the store out[slot][asset][path]
  // (Philox).  The words are consumed in counter order, so the loop runs over
  // groups of G slots whose G*A words fill NB whole Philox blocks: each word
  // comes from its block by a fixed index, with no per-word block test or
  // selection among the four.  The same words, steps and prices as step().
  __device__ __forceinline__ void store_philox(T* out, uint32_t npath) {
    constexpr int G = (A % 4 == 0) ? 1 : (A % 2 == 0) ? 2 : 4;
    constexpr int NB = G * A / 4;
    const int S = n_slots;
    int q = 0;
    uint32_t b = 0;
    for (; q + G <= S; q += G, b += NB) {
      uint32_t w[4 * NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) philox4x32_10(path, b + c, inst, 0u, k0, k1, &w[4 * c]);
#pragma unroll
      for (int j = 0; j < G; ++j) store_slot(out, npath, q + j, &w[j * A]);
    }
    if (q < S) {
      uint32_t w[4 * NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) philox4x32_10(path, b + c, inst, 0u, k0, k1, &w[4 * c]);
#pragma unroll
      for (int j = 0; j < G - 1; ++j)
        if (q + j < S) store_slot(out, npath, q + j, &w[j * A]);
    }
  }
  __device__ __forceinline__ void store_slot(T* out, uint32_t npath, int q, const uint32_t* wq) {
    uint32_t xw[A];
#pragma unroll
    for (int a = 0; a < A; ++a) xw[a] = wq[a];
    advance(xw, slotc[2 * q], slotc[2 * q + 1]);
#pragma unroll
    for (int a = 0; a < A; ++a) out[((size_t)q * A + a) * npath + path] = price(a);
  }

  // Generates slots up to s + WS - 1 (from the spot again on a backward
  // read) and keeps slots s .. s+WS-1 in the window.
  __device__ __forceinline__ void refill(T (&win)[kWindow], int s) {
    if (s < next_slot) {
#pragma unroll
      for (int a = 0; a < A; ++a) x[a] = T(0);
      next_slot = 0;
    }
    while (next_slot < s) { step(next_slot, nullptr, nullptr, 0); ++next_slot; }
    const int cnt = min(WS, n_slots - s);
#pragma unroll 1
    for (int j = 0; j < cnt; ++j) {
      step(s + j, nullptr, nullptr, 0);
#pragma unroll
      for (int a = 0; a < A; ++a) win[(j * A + a) & (kWindow - 1)] = price(a);
    }
    next_slot = s + cnt;
    base = s;
  }

  // The whole path (CAP > 0); nothing for the sliding window.  The loop
  // is written twice so that the Sobol one with the LDS table carries no
  // test of the other case.
  __device__ __forceinline__ void prime(Win& win) {
    if constexpr (CAP > 0) {
      if (RNG == 1 && use_lo) generate_all<true>(win);
      else generate_all<false>(win);
    }
  }
  // Software pipeline: the slot's scalar loads (step sizes; with the Sobol
  // table, the wave's high words) are issued one slot ahead, so a slot waits
  // only for its own LDS reads.  (Scalar and LDS loads share one counter and
  // scalar ones return out of order: the explicit wait ends this slot's
  // loads before the next slot's are issued.)
  template <bool LO>
  __device__ __forceinline__ void generate_all(Win& win) {
    if (n_slots <= 0) return;
    constexpr bool kTab = RNG == 1 && LO;
    uint32_t hw[A];
    T dt = slotc[0], sdt = slotc[1];
    if constexpr (kTab) {
#pragma unroll
      for (int a = 0; a < A; ++a) hw[a] = sobol_hi[a];
    }
#pragma unroll 1
    for (int q = 0; q < n_slots; ++q) {
      uint32_t xw[A];
      if constexpr (kTab) {
#pragma unroll
        for (int a = 0; a < A; ++a) xw[a] = lo[(uint32_t)(q * A + a) * 64u];
      }
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vector-memory and export counts untouched
      if constexpr (kTab) {
#pragma unroll
        for (int a = 0; a < A; ++a) xw[a] ^= hw[a];
      } else {
        words<false>(q, xw);
      }
      const T cdt = dt, csdt = sdt;
      const int nq = min(q + 1, n_slots - 1);
      dt = slotc[2 * nq];
      sdt = slotc[2 * nq + 1];
      if constexpr (kTab) {
#pragma unroll
        for (int a = 0; a < A; ++a) hw[a] = sobol_hi[nq * A + a];
      }
      advance(xw, cdt, csdt);
#pragma unroll
      for (int a = 0; a < A; ++a) win[(q * A + a) & (kWin - 1)] = price(a);
    }
  }

  __device__ __forceinline__ T read(Win& win, int slot, int a) {
    if constexpr (CAP > 0) {
      return win[uni(slot * A + a) & (CAP - 1)];
    } else {
      if (outside(slot, base, WS)) refill(win, slot);
      const int i = uni((slot - base) * A + a) & (kWindow - 1);
      return win[i];
    }
  }
  __device__ __forceinline__ T hist(int a, int day) const { return hist_value(histp, hist_first, n_hist, a, day); }
};

// Philox paths generated as a stream, for expressions whose reads never go
// back to an earlier slot (the host checks every instance's reads; the
// sliding window serves the others): each slot is generated once, when it
// is first read, and only the newest slot's prices are held, so there is no
// window to fill or index.  The words of a path are consumed in order, four
// per Philox block, from a per-thread buffer in LDS read at a uniform index.
// P paths per lane (P >= 1) share the wave-uniform work of every read and of
// the payoff's control flow (P = 2 halves the scalar instructions per
// path-date).  Each path's words, normals, steps and prices are those of
// GenSource, bit for bit.
template <typename T, int A, int P>
struct GenStream {
  using V = VecT<T, P>;
  using Mask = MaskT<P>;
  static constexpr int kWin = 1;
  using Win = char[1];
  T x[P][A];
  T cur[P][A];     // prices of slot `last`
  int last;        // newest generated slot (uniform), -1 before the first
  int left;        // words left in the buffer (uniform)
  uint32_t next_blk;
  // The Philox block in use (four words per path) sits in LDS, this
  // thread's word j of path e at wb[(j * P + e) * bs]: held in registers it
  // was part of the state every read carries, and the date loop and the
  // read's step kept that state in two register sets, copying it in and out
  // at every read.
  lwptr<uint32_t> wb;
  int bs;
  uint32_t path, k0, k1, inst;
  kptr<T> slotc;
  kptr<T> histp;
  int hist_first, n_hist;
  Model<T, A> M;

  __device__ __forceinline__ void restart() {
#pragma unroll
    for (int e = 0; e < P; ++e)
#pragma unroll
      for (int a = 0; a < A; ++a) x[e][a] = T(0);
    last = -1; left = 0; next_blk = 0;
  }
  __device__ __forceinline__ void init(const Args<T>& g, const InstDesc& d, uint32_t p, const T* l_own, bool own,
                                       lwptr<uint32_t> wbuf) {
    wb = wbuf + threadIdx.x;
    bs = (int)blockDim.x;
    path = p;
    k0 = g.k0; k1 = g.k1; inst = d.instance;
    M.load(g, d, l_own, own);
    slotc = K(g.rtab) + d.slot_off;
    histp = K(g.rtab) + d.hist_off;
    hist_first = d.hist_first; n_hist = d.n_hist;
    restart();
  }
  // the next word of each path
  __device__ __forceinline__ void next_word(uint32_t (&out)[P]) {
    if (left == 0) {
#pragma unroll
      for (int e = 0; e < P; ++e) {
        uint32_t o[4];
        philox4x32_10(path + (uint32_t)e, next_blk, inst, 0u, k0, k1, o);
#pragma unroll
        for (int q = 0; q < 4; ++q) wb[(q * P + e) * bs] = o[q];
      }
      ++next_blk;
      left = 4;
    }
    const int q = 4 - left;
#pragma unroll
    for (int e = 0; e < P; ++e) out[e] = wb[(q * P + e) * bs];
    --left;
  }
  // the next slot: GenSource::advance per path, then its prices
  __device__ __forceinline__ void step() {
    ++last;
    uint32_t xw[A][P];
#pragma unroll
    for (int a = 0; a < A; ++a) next_word(xw[a]);
    const T dt = slotc[2 * last], sdt = slotc[2 * last + 1];
#pragma unroll
    for (int e = 0; e < P; ++e) {
      T zs[A];
#pragma unroll
      for (int a = 0; a < A; ++a) zs[a] = Num<T>::normal_word_scaled(xw[a][e], sdt);
#pragma unroll
      for (int a = 0; a < A; ++a) {
        T xa = x[e][a] + M.dr[a] * dt;
#pragma unroll
        for (int k = 0; k <= a; ++k) xa = xa + M.C[a][k] * zs[k];
        x[e][a] = xa;
      }
#pragma unroll
      for (int a = 0; a < A; ++a) cur[e][a] = M.s0[a] * Num<T>::exps(x[e][a]);
    }
  }
  __device__ __forceinline__ V price_of(int a) const {
    if constexpr (P == 1) {
      return cur[0][a];
    } else {
      V r;
#pragma unroll
      for (int e = 0; e < P; ++e) r.v[e] = cur[e][a];
      return r;
    }
  }
  __device__ __forceinline__ void prime(Win&) {}
  // The newest slot, or the next one (one step, straight-line code: the
  // usual reads); any other slot by the loop below -- an earlier one, which
  // a checked expression never reads, from the spot again.
  __device__ __forceinline__ V read(Win&, int slot, int a) {
    if (slot != last) {
      if (slot == last + 1) {
        step();
      } else {
        if (slot < last) restart();
        while (last < slot) step();
      }
    }
    return price_of(a);
  }
  __device__ __forceinline__ V hist(int a, int day) const { return V(hist_value(histp, hist_first, n_hist, a, day)); }
};

// Sobol words of a wave's 64 points differ only in Gray-code bits 0..5 (bit 5
// also takes bit 6 of the point index): entry [w][b] of the block's LDS table
// is the XOR of dimension w's direction numbers selected by the bits of b, so
// a word is the wave's high part XOR one table read (64 distinct entries per
// wave: no bank conflicts).  Built by the whole block; false if the
// dimensions do not fit.
constexpr int kSobolLdsDims = 64;

// Each thread loads one dimension's six low direction numbers (one round
// trip, issued together) and writes four consecutive entries of it; a block
// of 256 threads covers 16 dimensions per pass.
template <typename T>
__device__ __forceinline__ bool sobol_lo_table(const Args<T>& g, uint32_t* tab) {
  if (!g.sobol_hi || g.sobol_dims > kSobolLdsDims) return false;
  const int per_pass = (int)blockDim.x >> 4;   // dimensions per pass
  for (int w = (int)threadIdx.x >> 4; w < g.sobol_dims; w += per_pass) {
    const uint32_t* v = g.sobol + (size_t)w * 32u;
    uint32_t d[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) d[b] = v[b];
    const int b0 = ((int)threadIdx.x & 15) * 4;
    uint32_t base = 0;   // XOR over bits 2..5 of b0
#pragma unroll
    for (int b = 2; b < 6; ++b) base ^= d[b] & (0u - (uint32_t)((b0 >> b) & 1));
    uint32_t* out = tab + w * 64 + b0;
    out[0] = base;
    out[1] = base ^ d[0];
    out[2] = base ^ d[1];
    out[3] = base ^ d[0] ^ d[1];
  }
  __syncthreads();
  return true;
}

// Reads stored prices [slot][asset][path] through the same kind of window;
// with P > 1 a lane holds paths path .. path+P-1 (path a multiple of P, the
// path count a multiple of P) and each entry is one P-wide load.
template <typename T, int A>
struct MemSource {
  using V = T;
  using Mask = bool;
  static constexpr int kWin = kWindow;
  using Win = T[kWindow];
  static constexpr int WS = kWindow / A;
  int base, n_slots;
  uint32_t path, n_paths;
  const T* paths;
  kptr<T> histp;
  int hist_first, n_hist;

  __device__ __forceinline__ void init(const Args<T>& g, const InstDesc& d, uint32_t p) {
    path = p; n_paths = d.n_paths; n_slots = d.n_slots; base = kNoWindow;
    paths = g.paths;
    histp = K(g.rtab) + d.hist_off;
    hist_first = d.hist_first; n_hist = d.n_hist;
  }
  // Loads slots s .. s+WS-1 (clamped) with WS * A independent loads.
  __device__ __forceinline__ void refill(Win& win, int s) {
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
  __device__ __forceinline__ void prime(Win&) {}
  __device__ __forceinline__ T read(Win& win, int slot, int a) {
    if (outside(slot, base, WS)) refill(win, slot);
    const int i = uni((slot - base) * A + a) & (kWindow - 1);
    return win[i];
  }
  __device__ __forceinline__ T hist(int a, int day) const { return hist_value(histp, hist_first, n_hist, a, day); }
};

// The same with P consecutive paths per lane (path a multiple of P, the path
// count a multiple of P): each window entry is one P-wide load, and the
// window lives in LDS laid out [entry][thread] so that a wave reads or
// writes one contiguous 64 * P * sizeof(T) bytes (no bank conflicts, and no
// register copies of a loop-carried window).
constexpr int kLdsWin = 4;   // window entries per lane

template <typename T, int A, int P>
struct MemSourceLds {
  using V = LaneVec<T, P>;
  using Mask = LaneMask<P>;
  static constexpr int kWin = kLdsWin;
  using Win = char[1];       // the window is in LDS
  static constexpr int WS = kLdsWin / A;
  int base, n_slots, stride;
  uint32_t path, n_paths;
  const T* paths;
  lwptr<T> lw;               // this lane's entry 0; entry i at lw + i * stride
  kptr<T> histp;
  int hist_first, n_hist;

  __device__ __forceinline__ void init(const Args<T>& g, const InstDesc& d, uint32_t p, lwptr<T> lds) {
    path = p; n_paths = d.n_paths; n_slots = d.n_slots; base = kNoWindow;
    paths = g.paths;
    stride = (int)blockDim.x * P;
    lw = lds + threadIdx.x * P;
    histp = K(g.rtab) + d.hist_off;
    hist_first = d.hist_first; n_hist = d.n_hist;
  }
  // Slots s .. s+WS-1 (clamped to the last): one 64-bit row offset, then
  // the others by adding the per-slot row stride (a window inside the path
  // needs no clamping).
  __device__ __forceinline__ void refill(int s) {
    const int last = n_slots - 1;
    const size_t row = (size_t)A * n_paths;   // elements per slot
    V x[WS * A];
    if (s + WS - 1 <= last) {
      const T* p0 = paths + (size_t)s * row + path;
#pragma unroll
      for (int j = 0; j < WS; ++j)
#pragma unroll
        for (int a = 0; a < A; ++a)
          x[j * A + a] = *reinterpret_cast<const V*>(p0 + (size_t)j * row + (size_t)a * n_paths);
    } else {
#pragma unroll
      for (int j = 0; j < WS; ++j) {
        const int q = min(s + j, last);
#pragma unroll
        for (int a = 0; a < A; ++a)
          x[j * A + a] = *reinterpret_cast<const V*>(paths + (size_t)q * row + (size_t)a * n_paths + path);
      }
    }
#pragma unroll
    for (int i = 0; i < WS * A; ++i)
#pragma unroll
      for (int e = 0; e < P; ++e) lw[i * stride + e] = x[i].v[e];
    base = s;
  }
  __device__ __forceinline__ void prime(Win&) {}
  __device__ __forceinline__ V read(Win&, int slot, int a) {
    if (outside(slot, base, WS)) refill(slot);
    const int i = uni((slot - base) * A + a);
    V r;
#pragma unroll
    for (int e = 0; e < P; ++e) r.v[e] = lw[i * stride + e];
    return r;
  }
  __device__ __forceinline__ V hist(int a, int day) const { return V(hist_value(histp, hist_first, n_hist, a, day)); }
};

// An observable of a model asset on a day: history for a day up to the
// simulation's start sim_from (the given price history, flat before its
// first day; without one, the spot), else the simulated price of the day's
// slot.  The grid is given by its first day when dense (else 0: the day map
// dm), its slot count and its horizon.  (A dense grid starts after sim_from,
// so its slot test also covers the history days.)
template <class Src>
__device__ __forceinline__ typename Src::V read_obs(Src& src, typename Src::Win& win, int dense_first,
                                                    int n_slots, int horizon, int sim_from, kptr<int32_t> dm,
                                                    int day, int asset) {
  int s;
  if (dense_first > 0) {
    s = min(day - dense_first, n_slots - 1);
  } else {
    if (day <= sim_from) return src.hist(asset, day);
    s = uni(dm[min(day, horizon)]);
  }
  return s < 0 ? src.hist(asset, day) : src.read(win, s, asset);
}

template <class Src>
__device__ __forceinline__ typename Src::V read_obs(Src& src, typename Src::Win& win, const InstDesc& D,
                                                    kptr<int32_t> dm, int day, int asset) {
  return read_obs(src, win, D.dense_first, D.n_slots, D.horizon, D.sim_from, dm, day, asset);
}

// ------------------------------------------------------- interpreter ------
template <typename T, int NR, class Src>
__device__ __forceinline__ T interpret(const Args<T>& g, const InstDesc& D, Src& src, int* frames) {
  T R[NR];
  T win[kWindow];
#pragma unroll
  for (int i = 0; i < NR; ++i) R[i] = T(0);
#pragma unroll
  for (int i = 0; i < kWindow; ++i) win[i] = T(0);
  kptr<int32_t> tt = K(g.itab) + D.tt_off;
  kptr<int32_t> dm = K(g.itab) + D.daymap_off;
  kptr<T> consts = K(g.consts);
  kptr<T> rt = K(g.rtab);
  kptr<int32_t> it = K(g.itab);
  kptr<uint32_t> code = K(reinterpret_cast<const uint32_t*>(g.code));
  int pc = 0, t0 = 0;
  int f_top = 0, f_rem = 0, f_t0 = 0, depth = 0;
  uint32_t w0 = (uint32_t)uni((int)code[0]);
  int imm = uni((int)code[1]);
  for (;;) {
    // prefetch the next instruction (the program ends with two HALTs)
    const uint32_t n0 = (uint32_t)uni((int)code[2 * pc + 2]);
    const int nimm = uni((int)code[2 * pc + 3]);
    const int op = w0 & 0xff, a = (w0 >> 16) & (NR - 1), b = (w0 >> 24) & (NR - 1);
    const int d = (w0 >> 8) & (NR - 1);
    const int ai = (w0 >> 16) & 0xff;  // asset / party-pair operand
    const int next = pc + 1;
    ++pc;
    if (op == OP_HALT) break;
    const T ra = R[a], rb = R[b];
    T v = T(0);
    switch (op) {
      case OP_CONST: v = consts[imm]; break;
      case OP_PARAM: v = rt[D.param_off + imm]; break;
      case OP_MODEL: v = read_obs(src, win, D, dm, tt[imm] + t0, ai); break;
      case OP_TEXPR: v = (T)(tt[imm] + t0); break;
      case OP_NOW: v = (T)D.t_now; break;
      case OP_PAYOFF: {
        const int day = min(max(tt[imm] + t0, 0), D.horizon);
        v = (T)it[D.sign_off + ai] * rt[D.disc_off + day];
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
      case OP_SEL: v = ra != T(0) ? rb : R[imm & (NR - 1)]; break;
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
    if (pc == next) {
      w0 = n0; imm = nimm;
    } else {
      w0 = (uint32_t)uni((int)code[2 * pc]);
      imm = uni((int)code[2 * pc + 1]);
    }
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
// Evaluator policy that interprets the loaded bytecode with an NR-entry
// register file.
template <int NR>
struct Interp {
  template <typename T, class Src>
  static __device__ __forceinline__ T run(const Args<T>& g, const InstDesc& D, Src& src, int* frames) {
    return interpret<T, NR>(g, D, src, frames);
  }
};

// P > 1 (stored or streamed paths): each lane evaluates P consecutive
// paths; a tile is then P * blockDim paths.
// STREAM: generated Philox paths as a stream (GenStream): for expressions
// that never read back to an earlier slot.
// FULL > 0: generated paths are held whole (GenSource's CAP; every
// instance of the launch has n_slots * A <= FULL).
// SINGLE: the launch prices one instrument in a fixed grid stride (no work
// queue, no instance order), so the batch machinery is compiled out.
// OWN: every launch of the kernel has each block factor its instrument's
// matrix (Args::factor is 1), so the prepared-factor branch is compiled out.
template <typename T, int RNG, int A, bool MEM, class Eval, int P = 1, int FULL = 0, bool SINGLE = false,
          bool OWN = false, bool STREAM = false>
__device__ __forceinline__ void mc_body(const Args<T>& g) {
  static_assert(!STREAM || (RNG == 0 && !MEM && FULL == 0), "streamed paths: Philox, generated, no whole path");
  static_assert(P == 1 || MEM || STREAM, "several generated paths per lane are streamed");
  static_assert(FULL == 0 || !MEM, "whole-path windows are for generated paths");
  // Wave priorities: the instruction arbiter favours older waves among equal
  // priorities, so a block that arrives a little later would have its set-up
  // (one thread's FP64 factorisation, the Sobol table, the barrier) starved by
  // older waves' tiles and finish last.  Set-up runs at the top priority and,
  // in a fixed stride, a wave with more tiles still to do outranks one on its
  // last, which evens out the waves' finishing times.
  __builtin_amdgcn_s_setprio(3);
  __shared__ double red[8];
  __shared__ int frames_all[4][3 * kMaxLoopDepth];
  __shared__ int item_s;
  __shared__ int last_s;
  int* frames = frames_all[threadIdx.x >> 6];
  // A single fused instrument: one thread of each block factors the
  // correlation matrix and makes the step coefficients from the factor and
  // the instrument's model into LDS (block 0 also reports whether the matrix
  // is positive definite) while the others build the Sobol table; after the
  // barrier that publishes both, every thread keeps the coefficients in
  // registers.  (The choice is an explicit flag, never a null test of an LDS
  // pointer: an LDS array may sit at address 0.)
  constexpr int kLA = A > 0 ? A * A : 1;
  T l_own[kLA + A] = {};   // the block's C (row-major), then dr: wave-uniform
  static_assert(!OWN || !MEM, "stored paths use the prepared factor");
  const bool own = OWN || (!MEM && g.factor != 0);
  __shared__ double chol_sh[kLA];
  __shared__ T coef_sh[kLA + A];
  if (own && threadIdx.x == 0) {
    const bool ok = chol_factor(K(g.chol_in), chol_sh, A);
    // (host-mapped memory, read after the host's wait on the launch's end
    // event, whose system-scope release publishes it)
    if (blockIdx.x == 0) g.status[0] = ok ? 0 : 1;
    kptr<T> m = K(g.rtab) + load_desc(g.desc, 0).model_off;
#pragma unroll
    for (int i = 0; i < A; ++i) {
#pragma unroll
      for (int j = 0; j < A; ++j) coef_sh[i * A + j] = Model<T, A>::diffusion_coef(chol_sh[i * A + j], m[A + i]);
      coef_sh[kLA + i] = Model<T, A>::drift_coef(m[i]);
    }
  }
  bool has_lo = false;
  lptr<uint32_t> lo_tab = nullptr;
  if constexpr (RNG == 1 && !MEM) {
    __shared__ uint32_t sob_lo[kSobolLdsDims * 64];
    has_lo = sobol_lo_table(g, sob_lo);   // ends with a barrier when it builds the table
    lo_tab = (lptr<uint32_t>)sob_lo;
  }
  if (own) {
    if (!has_lo) __syncthreads();
#pragma unroll
    for (int k = 0; k < kLA + A; ++k) l_own[k] = coef_sh[k];
  }
  lwptr<T> mem_win = nullptr;
  if constexpr (MEM && P > 1) {
    __shared__ __align__(16) T win_lds[kLdsWin * 256 * P];   // [entry][thread][P], blockDim <= 256
    mem_win = (lwptr<T>)win_lds;
  }
  // Work items come from the atomic queue (persistent batches) or in a
  // fixed grid stride (single instrument: the grid is at most what fits on
  // the chip, so per-block set-up is paid once per resident block).
  double bs = 0.0, bss = 0.0;   // fixed stride: this thread's sums over its tiles
  const bool queue = !SINGLE && g.queue != nullptr;
  int item = (int)blockIdx.x - (int)gridDim.x;
  for (;;) {
    if (queue) {
      if (threadIdx.x == 0) item_s = (int)atomicAdd(g.queue, 1u);
      __syncthreads();
      item = item_s;
      __syncthreads();
    } else {
      item += (int)gridDim.x;
    }
    if (item >= g.n_work) break;
    if (queue || item + (int)gridDim.x < g.n_work) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(1);
    // item -> (instance, tile): consecutive items cover one instance's tiles
    int2 wi = make_int2(0, item);
    if (!SINGLE && g.order) wi = make_int2(K(g.order)[item / g.tiles], item % g.tiles);
    const InstDesc D = load_desc(g.desc, wi.x);
    double s = 0.0, ss = 0.0;
    for (int r = 0; r < g.ppt; ++r) {
      // 64-bit: with n_paths close to 2^32 the last tile's lanes would wrap
      const uint64_t path0 =
          (((uint64_t)(uint32_t)wi.y * (uint32_t)g.ppt + (uint32_t)r) * blockDim.x + threadIdx.x) * P;
      const uint32_t p = path0 < D.n_paths ? (uint32_t)path0 : D.n_paths - P;
      VecT<T, P> v;
      if constexpr (MEM && P > 1) {
        MemSourceLds<T, A, P> src;
        src.init(g, D, p, mem_win);
        v = Eval::template run<T>(g, D, src, frames);
      } else if constexpr (MEM) {
        MemSource<T, A> src;
        src.init(g, D, p);
        v = Eval::template run<T>(g, D, src, frames);
      } else if constexpr (STREAM) {
        __shared__ uint32_t stream_words[4 * P * 256];   // [word][path][thread], blockDim <= 256 (4 KB per path)
        GenStream<T, A, P> src;
        src.init(g, D, p, l_own, own, (lwptr<uint32_t>)stream_words);
        v = Eval::template run<T>(g, D, src, frames);
      } else {
        GenSource<T, RNG, A, FULL> src;
        src.init(g, D, p, lo_tab, has_lo, l_own, own);
        v = Eval::template run<T>(g, D, src, frames);
      }
#pragma unroll
      for (int e = 0; e < P; ++e) {
        const uint64_t path = path0 + (uint32_t)e;
        if (path < D.n_paths) {
          const T ve = lane_elem(v, e);
          const double x = (double)ve;
          s += x; ss += x * x;
          if (g.payoff_out) g.payoff_out[path] = ve;
        }
      }
    }
    if (!queue) {            // one instrument: per-thread sums over its tiles, reduced once below
      bs += s; bss += ss;
      continue;
    }
    block_sum2(s, ss, red);
    // Queue: publish the tile's partial; the block that completes an
    // instance's last tile sums all its partials in tile order
    // (deterministic whichever block is last) and writes the result.
    // (release by every block: a write-back of this XCD's L2; acquire, an
    // L2 invalidation, only by the last one)
    if (threadIdx.x == 0) {
      g.partial[D.first_item + wi.y] = make_double2(s, ss);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      last_s = __hip_atomic_fetch_add(&g.done[wi.x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               D.n_tiles - 1u;
    }
    __syncthreads();
    if (last_s) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      double a = 0.0, b = 0.0;
      for (uint32_t i = threadIdx.x; i < D.n_tiles; i += blockDim.x) {
        const double2 q = g.partial[D.first_item + i];
        a += q.x; b += q.y;
      }
      block_sum2(a, b, red);
      if (threadIdx.x == 0) {
        g.result[wi.x] = make_double2(a, b);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");   // system scope: host-mapped memory
      }
    }
  }
  if (!queue) {
    // One block reduction and one partial per block; the finishing kernel
    // that follows on the stream sums the partials in block order.  (A
    // completion counter instead would serialize: device-scope atomics on
    // one address from every block of the chip cost about 20 ns each.)
    // Each thread's tiles are fixed by the stride, so the result is
    // deterministic.
    block_sum2(bs, bss, red);
    if (threadIdx.x == 0) g.partial[blockIdx.x] = make_double2(bs, bss);
  }
}

// Two-phase path generation: stored prices [slot][asset][path].
template <typename T, int RNG, int A>
__device__ __forceinline__ void pathgen_body(const Args<T>& g, T* out, uint32_t* wout, T* zout, uint32_t n_paths) {
  bool has_lo = false;
  lptr<uint32_t> lo_tab = nullptr;
  if constexpr (RNG == 1) {
    __shared__ uint32_t sob_lo[kSobolLdsDims * 64];
    has_lo = sobol_lo_table(g, sob_lo);
    lo_tab = (lptr<uint32_t>)sob_lo;
  }
  const uint64_t gpath = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gpath >= n_paths) return;
  const uint32_t path = (uint32_t)gpath;
  const InstDesc D = load_desc(g.desc, 0);
  GenSource<T, RNG, A> src;
  src.init(g, D, path, lo_tab, has_lo);
  if constexpr (RNG == 0) {
    if (!wout && !zout) {
      src.store_philox(out, n_paths);
      return;
    }
  }
  for (int q = 0; q < D.n_slots; ++q) {
    src.step(q, wout, zout, n_paths);
#pragma unroll
    for (int a = 0; a < A; ++a)
      out[((size_t)q * A + a) * n_paths + path] = src.price(a);
  }
}

}  // namespace eng
}  // namespace pmc
