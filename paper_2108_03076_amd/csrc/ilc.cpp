// Payoff language host side: S-expression reader, parser to the IL node set
// (Sec. 3 grammar; Coq ILExpr / ILTExpr / ILTExprZ of Sec. 5), type check over
// N + R + B (Fig. 3), register-machine bytecode encoder, and the grid planner
// (days a node can read under the loopif shifts of Fig. 3; re-indexing of
// Sec. 6.2).
#include "ilc.h"

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "../../include/pmc.h"

namespace pmc {
namespace {

// ---------------------------------------------------------------- reader ----
struct SExp {
  bool atom = false;
  std::string text;
  std::vector<SExp> items;
};

struct Reader {
  const char* s;
  size_t n, i = 0;
  std::string err;

  void skip() {
    while (i < n) {
      char c = s[i];
      if (c == ';') {
        while (i < n && s[i] != '\n') ++i;
      } else if (c == ' ' || c == '\t' || c == '\n' || c == '\r') {
        ++i;
      } else {
        break;
      }
    }
  }
  bool read(SExp& out, int depth) {
    if (depth > 4096) { err = "nesting too deep"; return false; }
    skip();
    if (i >= n) { err = "unexpected end of input"; return false; }
    if (s[i] == ')') { err = "unexpected ')'"; return false; }
    if (s[i] == '(') {
      ++i;
      out.atom = false;
      for (;;) {
        skip();
        if (i >= n) { err = "missing ')'"; return false; }
        if (s[i] == ')') { ++i; return true; }
        out.items.emplace_back();
        if (!read(out.items.back(), depth + 1)) return false;
      }
    }
    size_t j = i;
    while (i < n && s[i] != '(' && s[i] != ')' && s[i] != ' ' && s[i] != '\t' && s[i] != '\n' &&
           s[i] != '\r' && s[i] != ';')
      ++i;
    out.atom = true;
    out.text.assign(s + j, i - j);
    return true;
  }
};

bool parse_int(const std::string& t, int64_t& v) {
  if (t.empty()) return false;
  size_t k = (t[0] == '-' || t[0] == '+') ? 1 : 0;
  if (k == t.size()) return false;
  for (size_t q = k; q < t.size(); ++q)
    if (t[q] < '0' || t[q] > '9') return false;
  errno = 0;
  char* end = nullptr;
  long long x = std::strtoll(t.c_str(), &end, 10);
  if (errno != 0 || *end != 0) return false;
  v = x;
  return true;
}

bool parse_real(const std::string& t, double& v) {
  if (t.empty()) return false;
  errno = 0;
  char* end = nullptr;
  v = std::strtod(t.c_str(), &end);
  return *end == 0 && errno == 0;
}

// --------------------------------------------------------------- parser -----
struct Parser {
  Program& P;
  std::string err;
  int status = PMC_OK;

  explicit Parser(Program& p) : P(p) {}

  bool fail(int st, const std::string& m) {
    if (status == PMC_OK) { status = st; err = m; }
    return false;
  }

  int tvar_index(const std::string& name) {
    for (size_t i = 0; i < P.tvars.size(); ++i)
      if (P.tvars[i] == name) return (int)i;
    return -1;
  }

  // ILTExpr (allow_z = false) or ILTExprZ (allow_z = true) -> linear form
  bool texpr(const SExp& s, bool allow_z, Lin& out) {
    out.c = 0;
    out.k.assign(P.tvars.size(), 0);
    if (s.atom) {
      int64_t v;
      if (!parse_int(s.text, v) || v < 0) return fail(PMC_E_PARSE, "bad template numeral '" + s.text + "'");
      out.c = v;
      return true;
    }
    const auto& it = s.items;
    if (it.size() == 2 && it[0].atom && it[0].text == "tvar" && it[1].atom) {
      int v = tvar_index(it[1].text);
      if (v < 0) return fail(PMC_E_TENV, "template variable '" + it[1].text + "' is not declared");
      out.k[v] = 1;
      return true;
    }
    if (it.size() == 3 && it[0].atom && (it[0].text == "tplus" || (allow_z && it[0].text == "tplusz"))) {
      bool z = it[0].text == "tplusz";
      Lin a, b;
      if (!texpr(it[1], z, a) || !texpr(it[2], z, b)) return false;
      out.c = a.c + b.c;
      for (size_t v = 0; v < out.k.size(); ++v) out.k[v] = a.k[v] + b.k[v];
      return true;
    }
    if (allow_z && it.size() == 2 && it[0].atom && it[0].text == "int" && it[1].atom) {
      int64_t v;
      if (!parse_int(it[1].text, v)) return fail(PMC_E_PARSE, "bad int literal");
      out.c = v;
      return true;
    }
    return fail(PMC_E_PARSE, "bad template expression");
  }

  int intern_tt(const Lin& l) {
    for (size_t i = 0; i < P.tt.size(); ++i)
      if (P.tt[i] == l) return (int)i;
    P.tt.push_back(l);
    return (int)P.tt.size() - 1;
  }

  int intern_party(const std::string& s) {
    for (size_t i = 0; i < P.parties.size(); ++i)
      if (P.parties[i] == s) return (int)i;
    P.parties.push_back(s);
    return (int)P.parties.size() - 1;
  }

  int add(const Node& n) {
    P.nodes.push_back(n);
    return (int)P.nodes.size() - 1;
  }

  static bool binop_code(const std::string& h, uint8_t& op) {
    static const char* names[] = {"add", "sub", "mult", "div", "min", "max", "lt", "leq", "eq", "and", "or"};
    static const uint8_t codes[] = {OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_MIN, OP_MAX,
                                    OP_LT,  OP_LE,  OP_EQ,  OP_AND, OP_OR};
    for (int i = 0; i < 11; ++i)
      if (h == names[i]) { op = codes[i]; return true; }
    return false;
  }

  int expr(const SExp& s, int depth) {
    if (depth > 2000) { fail(PMC_E_UNSUPPORTED, "expression nested too deeply"); return -1; }
    if (s.atom) { fail(PMC_E_PARSE, "bare atom '" + s.text + "' where an expression is expected"); return -1; }
    if (s.items.empty() || !s.items[0].atom) { fail(PMC_E_PARSE, "form without a symbol head"); return -1; }
    const auto& it = s.items;
    const std::string& h = it[0].text;
    const size_t n = it.size();
    Node nd{};
    if (h == "now" && n == 1) { nd.kind = Node::NOW; nd.ty = Ty::N; return add(nd); }
    if (h == "real" && n == 2 && it[1].atom) {
      if (!parse_real(it[1].text, nd.real)) { fail(PMC_E_PARSE, "bad real literal"); return -1; }
      nd.kind = Node::REAL; nd.ty = Ty::R; return add(nd);
    }
    if (h == "nat" && n == 2 && it[1].atom) {
      int64_t v;
      if (!parse_int(it[1].text, v) || v < 0) { fail(PMC_E_PARSE, "bad nat literal"); return -1; }
      nd.kind = Node::NAT; nd.ty = Ty::N; nd.real = (double)v; return add(nd);
    }
    if (h == "bool" && n == 2 && it[1].atom && (it[1].text == "true" || it[1].text == "false")) {
      nd.kind = Node::BOOL; nd.ty = Ty::B; nd.real = it[1].text == "true" ? 1.0 : 0.0; return add(nd);
    }
    if (h == "t" && n == 2) {
      Lin l;
      if (!texpr(it[1], false, l)) return -1;
      nd.kind = Node::TEXPR; nd.ty = Ty::N; nd.tt = intern_tt(l); return add(nd);
    }
    if (h == "model" && n == 3 && it[1].atom) {
      Lin l;
      if (!texpr(it[2], true, l)) return -1;
      const std::string& lab = it[1].text;
      for (size_t a = 0; a < P.assets.size(); ++a)
        if (P.assets[a] == lab) {
          nd.kind = Node::MODEL; nd.obs = (int)a; nd.ty = Ty::R; nd.tt = intern_tt(l); return add(nd);
        }
      for (size_t q = 0; q < P.params.size(); ++q)
        if (P.params[q] == lab) {  // constant observable: the day does not matter
          nd.kind = Node::PARAM; nd.obs = (int)q; nd.ty = Ty::R; return add(nd);
        }
      fail(PMC_E_TYPE, "unknown observable '" + lab + "'");
      return -1;
    }
    if (h == "payoff" && n == 4 && it[2].atom && it[3].atom) {
      Lin l;
      if (!texpr(it[1], false, l)) return -1;
      int p1 = intern_party(it[2].text), p2 = intern_party(it[3].text);
      int pr = -1;
      for (size_t q = 0; q < P.pairs.size(); ++q)
        if (P.pairs[q].first == p1 && P.pairs[q].second == p2) pr = (int)q;
      if (pr < 0) { P.pairs.push_back({p1, p2}); pr = (int)P.pairs.size() - 1; }
      if (pr > 255) { fail(PMC_E_UNSUPPORTED, "more than 256 party pairs"); return -1; }
      nd.kind = Node::PAYOFF; nd.ty = Ty::R; nd.pair = pr; nd.tt = intern_tt(l); return add(nd);
    }
    if ((h == "if" && n == 4) || (h == "loopif" && n == 5)) {
      int c = expr(it[1], depth + 1);
      if (c < 0) return -1;
      int a = expr(it[2], depth + 1);
      if (a < 0) return -1;
      int b = expr(it[3], depth + 1);
      if (b < 0) return -1;
      if (P.nodes[c].ty != Ty::B) { fail(PMC_E_TYPE, h + " condition is not boolean"); return -1; }
      if (P.nodes[a].ty != P.nodes[b].ty) { fail(PMC_E_TYPE, h + " branches differ in type"); return -1; }
      nd.kind = h == "if" ? Node::IF : Node::LOOPIF;
      nd.ty = P.nodes[a].ty;
      nd.kid[0] = c; nd.kid[1] = a; nd.kid[2] = b;
      if (h == "loopif") {
        Lin l;
        if (!texpr(it[4], false, l)) return -1;
        nd.tt = intern_tt(l);
      }
      return add(nd);
    }
    if ((h == "neg" || h == "not") && n == 2) {
      int x = expr(it[1], depth + 1);
      if (x < 0) return -1;
      Ty t = P.nodes[x].ty;
      if (h == "neg" && t != Ty::R) { fail(PMC_E_TYPE, "neg of a non-real"); return -1; }
      if (h == "not" && t != Ty::B) { fail(PMC_E_TYPE, "not of a non-boolean"); return -1; }
      nd.kind = Node::UN; nd.op = h == "neg" ? OP_NEG : OP_NOT; nd.ty = t; nd.kid[0] = x;
      return add(nd);
    }
    uint8_t op;
    if (n == 3 && binop_code(h, op)) {
      int x = expr(it[1], depth + 1);
      if (x < 0) return -1;
      int y = expr(it[2], depth + 1);
      if (y < 0) return -1;
      Ty a = P.nodes[x].ty, b = P.nodes[y].ty;
      if (a != b) { fail(PMC_E_TYPE, h + " applied to different types"); return -1; }
      Ty r;
      switch (op) {
        case OP_ADD: case OP_MIN: case OP_MAX:
          if (a == Ty::B) { fail(PMC_E_TYPE, h + " of booleans"); return -1; }
          r = a; break;
        case OP_SUB: case OP_MUL: case OP_DIV:
          if (a != Ty::R) { fail(PMC_E_TYPE, h + " needs reals"); return -1; }
          r = Ty::R; break;
        case OP_LT: case OP_LE:
          if (a == Ty::B) { fail(PMC_E_TYPE, h + " of booleans"); return -1; }
          r = Ty::B; break;
        case OP_EQ: r = Ty::B; break;
        default:
          if (a != Ty::B) { fail(PMC_E_TYPE, h + " needs booleans"); return -1; }
          r = Ty::B; break;
      }
      nd.kind = Node::BIN; nd.op = op; nd.ty = r; nd.kid[0] = x; nd.kid[1] = y;
      return add(nd);
    }
    fail(PMC_E_PARSE, "unknown or malformed form '" + h + "'");
    return -1;
  }
};

// -------------------------------------------------------------- encoder -----
// Registers are allocated by depth with Sethi-Ullman ordering of binary
// operands: a node evaluated "at k" leaves its value in R[k] and may use
// R[k..k+need-1].
struct Encoder {
  Program& P;
  std::vector<int> need;
  int max_reg = 0, depth = 0, max_depth = 0;

  explicit Encoder(Program& p) : P(p), need(p.nodes.size(), 0) {}

  static bool is_leaf(const Node& n) {
    return n.kind != Node::IF && n.kind != Node::LOOPIF && n.kind != Node::UN && n.kind != Node::BIN;
  }

  int compute_need(int i) {
    const Node& n = P.nodes[i];
    int r = 1;
    switch (n.kind) {
      case Node::UN: r = compute_need(n.kid[0]); break;
      case Node::BIN: {
        int a = compute_need(n.kid[0]), b = compute_need(n.kid[1]);
        r = a == b ? a + 1 : std::max(a, b);
        break;
      }
      case Node::IF: {
        int c = compute_need(n.kid[0]), a = compute_need(n.kid[1]), b = compute_need(n.kid[2]);
        r = std::max({c, 1 + a, 2 + b});
        break;
      }
      case Node::LOOPIF: {
        int c = compute_need(n.kid[0]), a = compute_need(n.kid[1]), b = compute_need(n.kid[2]);
        r = std::max({2 + c, 3 + a, 2 + b});
        break;
      }
      default: break;
    }
    need[i] = r;
    return r;
  }

  int emit(uint8_t op, int d, int a, int b, int32_t imm) {
    Instr in;
    in.op = op; in.d = (uint8_t)d; in.a = (uint8_t)a; in.b = (uint8_t)b; in.imm = imm;
    P.code.push_back(in);
    return (int)P.code.size() - 1;
  }

  int const_index(double v) {
    for (size_t i = 0; i < P.consts.size(); ++i)
      if (std::memcmp(&P.consts[i], &v, sizeof v) == 0) return (int)i;
    P.consts.push_back(v);
    return (int)P.consts.size() - 1;
  }

  // code size of a subtree if emitted (to decide whether skipping it pays)
  int size(int i) const {
    const Node& n = P.nodes[i];
    switch (n.kind) {
      case Node::UN: return 1 + size(n.kid[0]);
      case Node::BIN: return 1 + size(n.kid[0]) + size(n.kid[1]);
      case Node::IF: return 3 + size(n.kid[0]) + size(n.kid[1]) + size(n.kid[2]);
      case Node::LOOPIF: return 9 + size(n.kid[0]) + size(n.kid[1]) + size(n.kid[2]);
      default: return 1;
    }
  }

  void gen(int i, int k) {
    const Node& n = P.nodes[i];
    max_reg = std::max(max_reg, k);
    switch (n.kind) {
      case Node::NOW: emit(OP_NOW, k, 0, 0, 0); break;
      case Node::REAL: case Node::NAT: case Node::BOOL:
        emit(OP_CONST, k, 0, 0, const_index(n.real)); break;
      case Node::TEXPR: emit(OP_TEXPR, k, 0, 0, n.tt); break;
      case Node::MODEL: emit(OP_MODEL, k, n.obs, 0, n.tt); break;
      case Node::PARAM: emit(OP_PARAM, k, 0, 0, n.obs); break;
      case Node::PAYOFF: emit(OP_PAYOFF, k, n.pair, 0, n.tt); break;
      case Node::UN:
        gen(n.kid[0], k);
        emit(n.op, k, k, 0, 0);
        break;
      case Node::BIN: {
        int x = n.kid[0], y = n.kid[1];
        if (need[x] >= need[y]) {
          gen(x, k); gen(y, k + 1);
          emit(n.op, k, k, k + 1, 0);
        } else {
          gen(y, k); gen(x, k + 1);
          emit(n.op, k, k + 1, k, 0);
        }
        break;
      }
      case Node::IF: {
        gen(n.kid[0], k);
        // Skip a branch when no lane needs it, unless it is a single leaf.
        bool skip_a = !is_leaf(P.nodes[n.kid[1]]);
        bool skip_b = !is_leaf(P.nodes[n.kid[2]]);
        int j1 = skip_a ? emit(OP_JNONE, kTrash, k, 0, 0) : -1;
        gen(n.kid[1], k + 1);
        if (skip_a) P.code[j1].imm = (int32_t)P.code.size();
        int j2 = skip_b ? emit(OP_JALL, kTrash, k, 0, 0) : -1;
        gen(n.kid[2], k + 2);
        if (skip_b) P.code[j2].imm = (int32_t)P.code.size();
        emit(OP_SEL, k, k, k + 1, k + 2);
        max_reg = std::max(max_reg, k + 2);
        break;
      }
      case Node::LOOPIF: {
        // R[k] result, R[k+1] done, R[k+2] condition / take / second branch,
        // R[k+3] first branch
        ++depth;
        max_depth = std::max(max_depth, depth);
        int c0 = const_index(0.0);
        emit(OP_CONST, k, 0, 0, c0);
        emit(OP_CONST, k + 1, 0, 0, c0);
        emit(OP_LOOP, kTrash, 0, 0, n.tt);
        gen(n.kid[0], k + 2);
        int jt = emit(OP_LTAKE, k + 2, k + 1, 0, 0);
        gen(n.kid[1], k + 3);
        emit(OP_LMERGE, k, k + 2, k + 3, 0);
        P.code[jt].imm = (int32_t)P.code.size();
        emit(OP_LDONE, k + 1, k + 2, 0, 0);
        int jn = emit(OP_LNEXT, kTrash, k + 1, 0, 0);
        gen(n.kid[2], k + 2);
        emit(OP_LELSE, k, k + 1, k + 2, 0);
        P.code[jn].imm = (int32_t)P.code.size();
        emit(OP_LEND, kTrash, 0, 0, 0);
        max_reg = std::max(max_reg, k + 3);
        --depth;
        break;
      }
    }
  }
};

}  // namespace

// Register allocation and bytecode emission for a typed node tree.
static int encode(Program& P, std::string& err) {
  P.code.clear();
  P.consts.clear();
  Encoder en(P);
  en.compute_need(P.root);
  en.gen(P.root, 0);
  en.emit(OP_HALT, kTrash, 0, 0, 0);
  en.emit(OP_HALT, kTrash, 0, 0, 0);   // padding: the interpreter prefetches pc + 1
  P.n_regs = en.max_reg + 1;
  P.loop_depth = en.max_depth;
  if (P.n_regs > kMaxRegs) {
    err = "expression needs " + std::to_string(P.n_regs) + " registers (limit " + std::to_string(kMaxRegs) + ")";
    return PMC_E_UNSUPPORTED;
  }
  if (P.loop_depth > kMaxLoopDepth) { err = "loopif nested deeper than 8"; return PMC_E_UNSUPPORTED; }
  return PMC_OK;
}

int compile(const char* text, size_t len, const std::vector<std::string>& assets,
            const std::vector<std::string>& params, const std::vector<std::string>& tvars,
            Program& out, std::string& err) {
  Program P;
  P.assets = assets; P.params = params; P.tvars = tvars;
  for (size_t i = 0; i < assets.size(); ++i)
    for (size_t j = 0; j < params.size(); ++j)
      if (assets[i] == params[j]) { err = "label '" + assets[i] + "' is both an asset and a parameter"; return PMC_E_ARG; }
  Reader rd{text, len};
  SExp s;
  if (!rd.read(s, 0)) { err = rd.err; return PMC_E_PARSE; }
  rd.skip();
  if (rd.i != rd.n) { err = "trailing input after expression"; return PMC_E_PARSE; }
  Parser ps(P);
  int root = ps.expr(s, 0);
  if (root < 0) { err = ps.err; return ps.status; }
  if (P.nodes[root].ty != Ty::R) { err = "payoff expression is not real-valued"; return PMC_E_TYPE; }
  P.root = root;
  const int st = encode(P, err);
  if (st != PMC_OK) return st;
  out = std::move(P);
  return PMC_OK;
}

// cutPayoff (Sec. 4.1): every payoff(t, p, q) becomes
// if(lt(t(t), now), 0.0, payoff(t, p, q)); the other constructors recurse.
int cut_payoff(const Program& in, Program& out, std::string& err) {
  Program P = in;
  const int n0 = (int)in.nodes.size();
  for (int i = 0; i < n0; ++i) {
    if (P.nodes[i].kind != Node::PAYOFF) continue;
    // keep the payoff as a new node; node i becomes the guard
    Node pay = P.nodes[i];
    P.nodes.push_back(pay);
    const int ipay = (int)P.nodes.size() - 1;
    Node tx{};
    tx.kind = Node::TEXPR; tx.ty = Ty::N; tx.tt = pay.tt;
    P.nodes.push_back(tx);
    const int itx = (int)P.nodes.size() - 1;
    Node now{};
    now.kind = Node::NOW; now.ty = Ty::N;
    P.nodes.push_back(now);
    const int inow = (int)P.nodes.size() - 1;
    Node lt{};
    lt.kind = Node::BIN; lt.op = OP_LT; lt.ty = Ty::B; lt.kid[0] = itx; lt.kid[1] = inow;
    P.nodes.push_back(lt);
    const int ilt = (int)P.nodes.size() - 1;
    Node zero{};
    zero.kind = Node::REAL; zero.ty = Ty::R; zero.real = 0.0;
    P.nodes.push_back(zero);
    const int izero = (int)P.nodes.size() - 1;
    Node g{};
    g.kind = Node::IF; g.ty = Ty::R; g.kid[0] = ilt; g.kid[1] = izero; g.kid[2] = ipay;
    P.nodes[i] = g;
  }
  const int st = encode(P, err);
  if (st != PMC_OK) return st;
  out = std::move(P);
  return PMC_OK;
}

// --------------------------------------------------------------- planner ----
namespace {
struct Walk {
  const Program& P;
  const std::vector<int32_t>& tt;
  int64_t hi_day = 0;
  std::vector<uint8_t>* mark = nullptr;  // second pass: days read for assets
  void go(int i, int64_t lo, int64_t hi) {
    const Node& n = P.nodes[i];
    switch (n.kind) {
      case Node::MODEL: {
        int64_t a = tt[n.tt] + lo, b = tt[n.tt] + hi;
        hi_day = std::max(hi_day, b);
        if (mark)
          for (int64_t d = std::max<int64_t>(a, 1); d <= b; ++d) (*mark)[d] = 1;
        break;
      }
      case Node::PAYOFF: hi_day = std::max(hi_day, tt[n.tt] + hi); break;
      case Node::LOOPIF: {
        int64_t c = tt[n.tt];
        go(n.kid[0], lo, hi + c);
        go(n.kid[1], lo, hi + c);
        go(n.kid[2], lo + c, hi + c);
        break;
      }
      case Node::IF: go(n.kid[0], lo, hi); go(n.kid[1], lo, hi); go(n.kid[2], lo, hi); break;
      case Node::UN: go(n.kid[0], lo, hi); break;
      case Node::BIN: go(n.kid[0], lo, hi); go(n.kid[1], lo, hi); break;
      default: break;
    }
  }
};
}  // namespace

int plan(const Program& p, const int32_t* tenv, Grid& g, std::string& err, int32_t sim_from) {
  const size_t nv = p.tvars.size();
  for (size_t v = 0; v < nv; ++v)
    if (tenv[v] < 0) { err = "template variable '" + p.tvars[v] + "' is negative"; return PMC_E_TENV; }
  g.tt.resize(p.tt.size());
  for (size_t i = 0; i < p.tt.size(); ++i) {
    int64_t x = p.tt[i].c;
    for (size_t v = 0; v < nv; ++v) x += p.tt[i].k[v] * (int64_t)tenv[v];
    if (x > PMC_MAX_HORIZON || x < -PMC_MAX_HORIZON) {
      err = "template expression value " + std::to_string(x) + " beyond the horizon limit";
      return PMC_E_HORIZON;
    }
    g.tt[i] = (int32_t)x;
  }
  Walk w{p, g.tt};
  w.go(p.root, 0, 0);
  if (w.hi_day > PMC_MAX_HORIZON) {
    err = "expression reads day " + std::to_string(w.hi_day) + " beyond the horizon limit";
    return PMC_E_HORIZON;
  }
  g.horizon = (int32_t)std::max<int64_t>(0, w.hi_day);
  std::vector<uint8_t> mark((size_t)g.horizon + 1, 0);
  w.mark = &mark;
  w.go(p.root, 0, 0);
  g.days.clear();
  g.daymap.assign((size_t)g.horizon + 1, -1);
  g.sim_from = std::max<int32_t>(0, sim_from);
  for (int32_t d = g.sim_from + 1; d <= g.horizon; ++d)
    if (mark[d]) {
      g.daymap[d] = (int32_t)g.days.size();
      g.days.push_back(d);
    }
  return PMC_OK;
}

// ------------------------------------------------------- streamed reads --
namespace {
struct StreamWalk {
  const Program& P;
  const Grid& g;
  int64_t budget;
  int64_t last = -1;
  bool ok = true;
  bool dense = false;
  // the slot a day reads (-1: history), as the engine maps it
  int64_t slot_of(int64_t day) const {
    if (day <= g.sim_from) return -1;
    if (dense) return std::min<int64_t>(day - g.days.front(), (int64_t)g.days.size() - 1);
    const int64_t s = g.daymap[(size_t)std::min<int64_t>(day, g.horizon)];
    return s;
  }
  void go(int i, int64_t t0) {
    if (!ok) return;
    if (--budget < 0) { ok = false; return; }
    const Node& n = P.nodes[i];
    switch (n.kind) {
      case Node::MODEL: {
        const int64_t s = slot_of(g.tt[n.tt] + t0);
        if (s < 0) break;
        if (s < last) { ok = false; return; }
        last = s;
        break;
      }
      case Node::UN: go(n.kid[0], t0); break;
      case Node::BIN: go(n.kid[0], t0); go(n.kid[1], t0); break;
      case Node::IF: go(n.kid[0], t0); go(n.kid[1], t0); go(n.kid[2], t0); break;
      case Node::LOOPIF: {
        const int64_t count = g.tt[n.tt];
        for (int64_t k = 0; k <= count && ok; ++k) {
          go(n.kid[0], t0 + k);
          go(n.kid[1], t0 + k);
          if (k == count) go(n.kid[2], t0 + k);
        }
        break;
      }
      default: break;
    }
  }
};
}  // namespace

bool stream_reads(const Program& p, const Grid& g, int64_t max_visits) {
  StreamWalk w{p, g, max_visits};
  w.dense = !g.days.empty() && g.days.back() - g.days.front() + 1 == (int32_t)g.days.size();
  w.go(p.root, 0);
  return w.ok;
}

// ------------------------------------------------- fused window cost model --
int64_t fused_generation_cost(const Program& p, const Grid& g, int n_assets, int64_t max_events) {
  // Replays the bytecode's uniform control flow with every branch and every
  // loop iteration taken, and the fused kernel's window policy: a read of
  // slot s outside [base, base + ws) refills the window at s, generating
  // forward from the last generated slot, or from slot 0 if s is behind it.
  const int ws = std::max(1, kWindow / std::max(1, n_assets));
  int64_t generated = 0, events = 0;
  int64_t base = -1, next_gen = 0;
  struct Frame { int top; int64_t rem, t0; };
  std::vector<Frame> st;
  int64_t t0 = 0;
  int pc = 0;
  const int n = (int)p.code.size();
  while (pc < n) {
    if (++events > max_events) return -1;
    const Instr& in = p.code[pc++];
    switch (in.op) {
      case OP_HALT: return generated;
      case OP_MODEL: {
        int64_t day = g.tt[in.imm] + t0;
        if (day <= g.sim_from || day > g.horizon) break;
        int64_t s = g.daymap[day];
        if (s < 0) break;
        if (base >= 0 && s >= base && s < base + ws) break;
        if (s < next_gen) next_gen = 0;        // restart from the spot
        int64_t end = std::min<int64_t>((int64_t)g.days.size(), s + ws);
        generated += end - next_gen;
        next_gen = end;
        base = s;
        break;
      }
      case OP_LOOP: st.push_back({pc, g.tt[in.imm], t0}); break;
      case OP_LNEXT:
        if (st.back().rem == 0) break;
        st.back().rem--; t0++; pc = st.back().top;
        break;
      case OP_LEND: t0 = st.back().t0; st.pop_back(); break;
      default: break;   // JNONE / JALL / LTAKE fall through: all branches taken
    }
  }
  return generated;
}

}  // namespace pmc
