// Drives the contract-language front end (lexer, parser, the compilation to
// payoff-language text) and then the payoff loader on its output, over
// contract texts read from stdin, one per line, for sanitizer builds (host
// code only).  Prints one status line per input: the status of
// pmc_contract_compile, then (for compiled contracts) that of loading the
// resulting payoff.  The context-dependent parts of the library are
// replaced by the two functions below.
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "../include/pmc.h"
#include "ctx.h"
#include "ilc.h"

namespace pmc {
int ctx_fail(pmc_ctx*, int status, const std::string&) { return status; }
}  // namespace pmc

// pmc_payoff_load without a device: the loader's parse, type check and
// encoding of the text, with the labels given.
extern "C" int pmc_payoff_load(pmc_ctx*, const char* il_text, size_t len, const char* const* asset_labels,
                               int n_assets, const char* const* param_labels, int n_params,
                               const char* const* tvar_names, int n_tvars, pmc_payoff** out) {
  std::vector<std::string> a(asset_labels, asset_labels + n_assets), p(param_labels, param_labels + n_params),
      t(tvar_names, tvar_names + n_tvars);
  pmc::Program prog;
  std::string err;
  *out = nullptr;
  return pmc::compile(il_text, len, a, p, t, prog, err);
}

int main() {
  const char* assets[] = {"S", "S1", "S2", "S3"};
  const char* params[] = {"K", "B", "K1", "K2"};
  const char* tvars[] = {"T", "N", "a", "b"};
  std::string line;
  long n = 0, compiled = 0, loaded = 0;
  while (std::getline(std::cin, line)) {
    ++n;
    size_t len = 0;
    int st = pmc_contract_compile(line.data(), line.size(), nullptr, 0, &len);
    int ld = -1;
    if (st == PMC_OK) {
      ++compiled;
      std::string il(len + 1, '\0');
      size_t len2 = 0;
      if (pmc_contract_compile(line.data(), line.size(), &il[0], il.size(), &len2) != PMC_OK || len2 != len) {
        std::printf("compile not repeatable\n");
        return 2;
      }
      pmc_payoff* p = nullptr;
      ld = pmc_contract_load(nullptr, line.data(), line.size(), assets, 4, params, 4, tvars, 4, &p);
      if (ld == PMC_OK) ++loaded;
    }
    std::printf("%d %d\n", st, ld);
  }
  std::fprintf(stderr, "%ld inputs, %ld compiled, %ld loaded\n", n, compiled, loaded);
  return 0;
}
