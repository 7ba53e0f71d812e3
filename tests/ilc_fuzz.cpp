// Drives the host-side payoff loader (parse, type check, encode, cutPayoff,
// grid planning, fused-window cost) over IL texts read from stdin, one per
// line, for sanitizer builds.  Prints one status line per input.
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "ilc.h"

int main() {
  std::string line;
  const std::vector<std::string> assets = {"S", "S1", "S2", "S3"};
  const std::vector<std::string> params = {"K", "B"};
  const std::vector<std::string> tvars = {"T", "N", "a", "b"};
  long n = 0, ok = 0;
  while (std::getline(std::cin, line)) {
    ++n;
    pmc::Program p;
    std::string err;
    int st = pmc::compile(line.data(), line.size(), assets, params, tvars, p, err);
    if (st == 0) {
      ++ok;
      pmc::Program c;
      st = pmc::cut_payoff(p, c, err);
      const int32_t tenvs[3][4] = {{3, 2, 1, 0}, {0, 0, 0, 0}, {40, 4, 5, 2}};
      for (auto& t : tenvs) {
        pmc::Grid g;
        if (pmc::plan(p, t, g, err) == 0) (void)pmc::fused_generation_cost(p, g, 3, 100000);
        pmc::Grid gc;
        if (st == 0 && pmc::plan(c, t, gc, err) == 0 && gc.days != g.days) {
          std::printf("grid mismatch after cut\n");
          return 2;
        }
      }
    }
    std::printf("%d\n", st);
  }
  std::fprintf(stderr, "%ld inputs, %ld loaded\n", n, ok);
  return 0;
}
