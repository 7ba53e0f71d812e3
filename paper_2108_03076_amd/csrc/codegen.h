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

#include "ilc.h"
#include "kernels.h"

namespace pmc {

// Source of the generated payoff evaluator for one program.
std::string generate_payoff(const Program& P);

// Compiled kernels of one payoff, keyed by (device, precision, rng, assets,
// memory source, paths per lane).  Owned by the payoff object.
class JitCache {
 public:
  ~JitCache();
  // Returns the kernel for the variant, compiling it on first use.
  // lanes > 1 (paths per lane) is for the memory source only.
  int get(const Program& P, int device, int precision, int rng, int n_assets, bool from_memory,
          hipFunction_t* out, std::string& err, int lanes = 1);

 private:
  std::mutex mu_;
  std::map<std::string, std::pair<hipModule_t, hipFunction_t>> k_;
  std::string src_;  // generated payoff source (built once)
};

}  // namespace pmc
