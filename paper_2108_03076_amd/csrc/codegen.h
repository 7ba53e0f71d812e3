// Payoff code generation: the payoff expression is translated to a HIP device
// function (the code-generation route of the paper's Sec. 6, where each
// compiled contract becomes a target-language function that the pricing
// engine is instantiated with) and compiled at run time with hipRTC into the
// same Monte Carlo kernel body the interpreter uses.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ilc.h"
#include "kernels.h"

namespace pmc {

// Source of the generated payoff evaluator for one program: generic (G null:
// template values, grid, loop shifts and tables read at run time), or for
// the one template environment whose grid is G (its values constants; with
// `fixed`, loop iterations written out and the held path read at fixed
// registers).
std::string generate_payoff(const Program& P, const Grid* G, bool fixed);

// Statements generate_payoff writes for node i under grid G (each loopif
// iteration written out), capped at cap; kernels for one template
// environment are generated only up to kMaxUnrolled.
int64_t unrolled_size(const Program& P, const Grid& G, int i, int64_t cap);
constexpr int64_t kMaxUnrolled = 1024;

// Compiled kernels of one payoff, keyed by (device, precision, rng, assets,
// memory source, paths per lane, whole-path capacity, single instrument,
// own factorisation, template environment).  Owned by the payoff object.
class JitCache {
 public:
  ~JitCache();
  // Returns the kernel for the variant, compiling it on first use.
  // lanes > 1 (paths per lane) is for the memory source and for streamed
  // paths; full > 0 (a power of two, at most 32 values) holds each generated
  // path whole; stream: Philox paths generated as a stream (expressions
  // whose reads never go back to an earlier slot); tenv:
  // the one template environment every instance of the launch has, for a
  // kernel generated for it; null for the generic kernel.  single: the
  // launch prices one instrument without a work queue or instance order,
  // and the kernel leaves out the batch machinery.  own: every launch has
  // each block factor the correlation matrix itself (Args::factor = 1), and
  // the kernel leaves out the prepared-factor branch.
  int get(const Program& P, int device, int precision, int rng, int n_assets, bool from_memory,
          hipFunction_t* out, std::string& err, int lanes = 1, int full = 0, const int32_t* tenv = nullptr,
          bool single = false, bool own = false, bool stream = false);
 private:
  // The cache key of a variant; g and spec receive the grid and whether the
  // kernel is generated for that one template environment.
  static std::string variant_key(const Program& P, int device, int precision, int rng, int n_assets, bool mem,
                                 int lanes, int full, const int32_t* tenv, bool single, bool own, bool stream,
                                 Grid& g, bool& spec);
  // hipRTC compile and module load of one variant; waves > 0 asks for that
  // many waves per SIMD.
  int compile(const std::string& src, int precision, int rng, int n_assets, bool mem, int lanes, int full,
              bool single, bool own, bool stream, int waves, hipModule_t* mod, hipFunction_t* fn,
              std::string& err);
  std::mutex mu_;
  std::map<std::string, std::pair<hipModule_t, hipFunction_t>> k_;
  std::string src_;  // generic generated payoff source (built once)
};

}  // namespace pmc
