// Bytecode and per-instance descriptors shared by the host encoder and the
// device interpreter.  Plain structs only (host and device compile this).
#pragma once
#include <stdint.h>

namespace pmc {

// One interpreter instruction: 8 bytes, fetched by the whole wavefront at a
// uniform program counter (scalar loads).  Registers are per-lane values of
// the working precision; register kTrash absorbs results of instructions
// that write nothing.
struct Instr {
  uint8_t op;   // Op
  uint8_t d;    // destination register
  uint8_t a;    // first operand register / asset / party pair
  uint8_t b;    // second operand register
  int32_t imm;  // immediate: const-pool index, time-table index, jump target
};

enum Op : uint8_t {
  OP_HALT = 0,   // result in R[a]
  OP_CONST,      // R[d] = consts[imm]
  OP_PARAM,      // R[d] = params[imm]
  OP_MODEL,      // R[d] = observable asset a on day tt[imm] + t0
  OP_TEXPR,      // R[d] = tt[imm] + t0                       (N value)
  OP_NOW,        // R[d] = t_now                              (N value)
  OP_PAYOFF,     // R[d] = sign[a] * disc[tt[imm] + t0]
  OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_MIN, OP_MAX,
  OP_LT, OP_LE, OP_EQ, OP_AND, OP_OR,
  OP_NEG,        // R[d] = -R[a]
  OP_NOT,        // R[d] = !R[a]
  OP_SEL,        // R[d] = R[a] ? R[b] : R[imm]
  OP_JNONE,      // if no lane has R[a] != 0: pc = imm
  OP_JALL,       // if every lane has R[a] != 0: pc = imm
  OP_LOOP,       // push loop frame: top = pc+1, rem = tt[imm], saved t0
  OP_LTAKE,      // R[d] = !R[a] && R[d]   (take = not done and cond);
                 // if no lane takes: pc = imm
  OP_LMERGE,     // R[d] = R[a] ? R[b] : R[d]   (res = take ? branch : res)
  OP_LDONE,      // R[d] = R[d] || R[a]         (done |= take)
  OP_LNEXT,      // if every lane has R[a] (done): pc = imm; else if rem == 0
                 // fall through (second branch at t0); else rem--, t0++, pc = top
  OP_LELSE,      // R[d] = R[a] ? R[d] : R[b]   (res = done ? res : else)
  OP_LEND,       // t0 = saved t0; pop frame
  OP_COUNT
};

// Register files hold 8 or 32 values per lane (the kernel is specialised by
// the program's register count); indices are masked to the file size, so the
// write sink 31 lands on the file's last register in either size.
constexpr int kMaxRegs = 31;           // user registers R[0 .. kMaxRegs-1]
constexpr int kTrash = 31;             // write sink
constexpr int kRegFile = 32;           // largest register file
constexpr int kMaxLoopDepth = 8;
constexpr int kWindow = 16;            // cached path values per lane

// Everything one instance (one template environment, parameter set and
// model) needs; offsets index the packed tables of a launch.
struct InstDesc {
  int32_t tt_off;      // int table: folded template values (time table)
  int32_t sign_off;    // int table: party-pair signs (+1, -1, 0)
  int32_t daymap_off;  // int table: slot of each day 0..H (-1 for day 0)
  int32_t horizon;     // H: largest day read
  int32_t n_slots;     // simulated days
  int32_t t_now;       // value of (now)
  int32_t disc_off;    // real table: d(day), day 0..H
  int32_t slot_off;    // real table: (dt, sqrt dt) per slot
  int32_t param_off;   // real table: parameter observables
  int32_t model_off;   // real table: mu[A], sigma[A], spot[A]
  int32_t chol_off;    // double table: lower Cholesky factor, A x A
  uint32_t instance;   // Philox counter word 2
  uint32_t n_paths;
  uint32_t n_tiles;    // work items of this instance
  int32_t first_item;  // index of its first partial-sum slot
  int32_t dense_first; // > 0: the slots are the consecutive days dense_first ..
                       // dense_first + n_slots - 1 (no day map lookup needed)
  int32_t sim_from;    // the day the simulation starts from: days up to it
                       // are history, later days are simulated slots
  int32_t hist_off;    // real table: history [A][n_hist] (days hist_first ..
                       // hist_first + n_hist - 1; the spot alone if none given)
  int32_t hist_first;  // day of the history's first entry
  int32_t n_hist;      // history entries per asset (>= 1)
};

}  // namespace pmc
