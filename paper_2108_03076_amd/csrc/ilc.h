// Host side of the payoff language: reader, type check, bytecode encoder and
// the per-template-environment grid planner.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "pmc_device.h"

namespace pmc {

enum class Ty : uint8_t { N, R, B };

// A template expression folded to linear form: c + sum_v k[v] * delta(v).
struct Lin {
  int64_t c = 0;
  std::vector<int64_t> k;  // one coefficient per template variable
  bool operator==(const Lin& o) const { return c == o.c && k == o.k; }
};

struct Node {
  enum Kind : uint8_t { NOW, REAL, NAT, BOOL, TEXPR, MODEL, PARAM, PAYOFF, IF, LOOPIF, UN, BIN } kind;
  uint8_t op = 0;   // Op for UN / BIN
  Ty ty = Ty::R;
  double real = 0;  // REAL, NAT and BOOL values (as numbers)
  int obs = -1;     // MODEL: asset index; PARAM: parameter index
  int pair = -1;    // PAYOFF: party pair
  int tt = -1;      // time-table entry (TEXPR, MODEL, PAYOFF, LOOPIF count)
  int kid[3] = {-1, -1, -1};
};

struct Program {
  std::vector<std::string> assets, params, tvars, parties;
  std::vector<std::pair<int, int>> pairs;  // (from, to) party indices of payoff nodes
  std::vector<Node> nodes;
  int root = -1;
  std::vector<Lin> tt;       // distinct template expressions
  std::vector<Instr> code;
  std::vector<double> consts;
  int n_regs = 0;
  int loop_depth = 0;
};

// Parse, type-check and encode.  Returns a pmc_status; err gets the reason.
int compile(const char* text, size_t len, const std::vector<std::string>& assets,
            const std::vector<std::string>& params, const std::vector<std::string>& tvars,
            Program& out, std::string& err);

// cutPayoff of Sec. 4.1 applied to a compiled program (re-encoded).
int cut_payoff(const Program& in, Program& out, std::string& err);

// Per-template-environment plan: folded time table and simulated grid.
struct Grid {
  std::vector<int32_t> tt;      // value of every time-table entry
  std::vector<int32_t> days;    // simulated days (sorted, > sim_from)
  std::vector<int32_t> daymap;  // day 0..horizon -> slot or -1
  int32_t horizon = 0;
  int32_t sim_from = 0;         // last history day: the simulation starts from it
};
// sim_from: the last day of a given price history (days up to it are not
// simulated); 0 without one.
int plan(const Program& p, const int32_t* tenv, Grid& g, std::string& err, int32_t sim_from = 0);

// True if, evaluated with every branch taken and every loop iteration run
// (in the order the compiled payoff evaluates its nodes), the expression
// reads the simulated slots in non-decreasing order: then a path can be
// generated as a stream, each slot once and only the newest one held.  False
// also when the walk would exceed max_visits node visits.
bool stream_reads(const Program& p, const Grid& g, int64_t max_visits);

// Estimated number of generated slots per path when the fused interpreter
// serves the expression's reads through its kWindow-entry window (restarting
// generation on a backward read), assuming every branch and iteration runs.
// Returns -1 if the trace exceeds max_events.
int64_t fused_generation_cost(const Program& p, const Grid& g, int n_assets, int64_t max_events);

}  // namespace pmc
