// Contract language (CL) front end: reader for the contract syntax of
// Sec. 2 (Fig. 1, with template expressions in translate and ifWithin) and
// the compilation of Sec. 4 to the payoff language: tau_e for expressions
// and tau_c for contracts, with the starting time t0 accumulated through
// translate by the smart constructor for template addition.  The result is
// payoff-language text in the loader's syntax (include/pmc.h), which
// pmc_contract_load hands to pmc_payoff_load.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pmc.h"
#include "ctx.h"

namespace {

// ------------------------------------------------------------- lexer ------
struct Tok {
  enum Kind { END, ID, NUM, PUNCT } kind = END;
  std::string text;
  size_t pos = 0;
};

struct Lexer {
  const char* s;
  size_t n, i = 0;
  std::vector<Tok> toks;
  std::string err;

  bool run() {
    while (true) {
      while (i < n && (std::isspace((unsigned char)s[i]) || s[i] == ';')) {
        if (s[i] == ';') {   // a comment runs to the end of the line
          while (i < n && s[i] != '\n') ++i;
        } else {
          ++i;
        }
      }
      Tok t;
      t.pos = i;
      if (i >= n) { toks.push_back(t); return true; }
      const char c = s[i];
      if (std::isalpha((unsigned char)c) || c == '_') {
        size_t j = i;
        while (j < n && (std::isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
        t.kind = Tok::ID;
        t.text.assign(s + i, j - i);
        i = j;
      } else if (std::isdigit((unsigned char)c) || (c == '.' && i + 1 < n && std::isdigit((unsigned char)s[i + 1]))) {
        size_t j = i;
        while (j < n && (std::isdigit((unsigned char)s[j]) || s[j] == '.')) ++j;
        if (j < n && (s[j] == 'e' || s[j] == 'E')) {
          size_t k = j + 1;
          if (k < n && (s[k] == '+' || s[k] == '-')) ++k;
          if (k < n && std::isdigit((unsigned char)s[k])) {
            j = k;
            while (j < n && std::isdigit((unsigned char)s[j])) ++j;
          }
        }
        t.kind = Tok::NUM;
        t.text.assign(s + i, j - i);
        i = j;
      } else {
        static const char* two[] = {"<=", ">=", "==", "&&", "||"};
        t.kind = Tok::PUNCT;
        t.text.assign(1, c);
        for (const char* op : two)
          if (i + 1 < n && s[i] == op[0] && s[i + 1] == op[1]) t.text = op;
        if (c == 0 || !std::strchr("()[],+-*/<>!=&|", c) || t.text == "=" || t.text == "&" || t.text == "|") {
          err = "unexpected character '" + std::string(1, c) + "' at offset " + std::to_string(i);
          return false;
        }
        i += t.text.size();
      }
      toks.push_back(t);
    }
  }
};

// --------------------------------------------------- template expressions --
// TExp (Fig. 1: a numeral or a template variable) and the payoff language's
// ILTExpr / ILTExprZ: numerals n >= 0, integer literals, variables and the
// two additions.
struct TE {
  enum Kind { NAT, INT, VAR, PLUS, PLUSZ } kind = NAT;
  int64_t val = 0;
  std::string var;
  std::shared_ptr<TE> a, b;
  bool numeral() const { return kind == NAT || kind == INT; }
  bool z() const { return kind == INT || kind == PLUSZ; }   // an ILTExprZ only
};
using TP = std::shared_ptr<TE>;

TP nat(int64_t n) { auto t = std::make_shared<TE>(); t->kind = TE::NAT; t->val = n; return t; }
TP integer(int64_t n) {
  auto t = std::make_shared<TE>();
  t->kind = n >= 0 ? TE::NAT : TE::INT;
  t->val = n;
  return t;
}

// The smart constructor of Sec. 4: two numerals are added; otherwise the
// syntactic addition (ILTPlus of two ILTExpr, else ILTPlusZ).  Adding the
// numeral 0 is the identity (the compiled form Example 3 prints).
TP tplus(const TP& x, const TP& y) {
  if (x->numeral() && y->numeral()) {
    const int64_t v = x->val + y->val;
    auto t = std::make_shared<TE>();
    t->kind = (x->kind == TE::NAT && y->kind == TE::NAT) ? TE::NAT : TE::INT;
    t->val = v;
    return t;
  }
  if (x->kind == TE::NAT && x->val == 0 && !y->z()) return y;
  if (y->kind == TE::NAT && y->val == 0 && !x->z()) return x;
  auto t = std::make_shared<TE>();
  t->kind = (x->z() || y->z()) ? TE::PLUSZ : TE::PLUS;
  t->a = x;
  t->b = y;
  return t;
}

void put_te(std::string& o, const TE& t) {
  switch (t.kind) {
    case TE::NAT: o += std::to_string(t.val); break;
    case TE::INT: o += "(int " + std::to_string(t.val) + ")"; break;
    case TE::VAR: o += "(tvar " + t.var + ")"; break;
    case TE::PLUS: o += "(tplus "; put_te(o, *t.a); o += " "; put_te(o, *t.b); o += ")"; break;
    case TE::PLUSZ: o += "(tplusz "; put_te(o, *t.a); o += " "; put_te(o, *t.b); o += ")"; break;
  }
}

// ---------------------------------------------------------- the compiler --
// A recursive-descent reader that compiles while it reads: tau_e(e, t0)
// and tau_c(c, t0) are syntax-directed, so each construct's payoff text is
// produced from its parts' texts with the t0 in force at that point.
// Times and observation offsets are days: naturals of at most 31 bits (the
// payoff language's are 32-bit), so sums of nested translations stay far
// inside 64 bits.
bool day_numeral(const std::string& s, int64_t& v) {
  if (s.empty() || s.size() > 10 || s.find_first_not_of("0123456789") != std::string::npos) return false;
  v = std::strtoll(s.c_str(), nullptr, 10);
  return v <= 0x7fffffff;
}

// Nesting of contracts and expressions the compiler follows (it recurses
// once per level).
constexpr int kMaxNesting = 1000;

struct Compiler {
  const std::vector<Tok>& tk;
  size_t p = 0;
  std::string err;
  int depth = 0;
  // one level deeper for the lifetime of the guard; ok is false beyond the limit
  struct Deeper {
    Compiler& c;
    bool ok;
    explicit Deeper(Compiler& cc) : c(cc), ok(++cc.depth <= kMaxNesting) {}
    ~Deeper() { --c.depth; }
  };

  const Tok& cur() const { return tk[p]; }
  bool is(const char* punct) const { return cur().kind == Tok::PUNCT && cur().text == punct; }
  bool is_id(const char* id) const { return cur().kind == Tok::ID && cur().text == id; }
  bool fail(const std::string& m) {
    if (err.empty()) err = m + " at offset " + std::to_string(cur().pos);
    return false;
  }
  bool expect(const char* punct) {
    if (!is(punct)) return fail(std::string("expected '") + punct + "'");
    ++p;
    return true;
  }
  bool ident(std::string& out) {
    if (cur().kind != Tok::ID) return fail("expected a name");
    out = cur().text;
    ++p;
    return true;
  }

  // TExp: a numeral or a template variable
  bool texp(TP& out) {
    if (cur().kind == Tok::NUM) {
      int64_t v;
      if (!day_numeral(cur().text, v)) return fail("a time must be a natural number below 2^31");
      out = nat(v);
      ++p;
      return true;
    }
    if (cur().kind == Tok::ID) {
      auto t = std::make_shared<TE>();
      t->kind = TE::VAR;
      t->var = cur().text;
      out = t;
      ++p;
      return true;
    }
    return fail("expected a time (a natural number or a template variable)");
  }

  // --- contracts: tau_c(c, t0)
  bool contract(const TP& t0, std::string& o) {
    const Deeper d(*this);
    if (!d.ok) return fail("contract nested too deeply");
    if (cur().kind != Tok::ID) return fail("expected a contract");
    const std::string k = cur().text;
    ++p;
    if (k == "zero") {
      o = "(real 0.0)";
      return true;
    }
    if (k == "transfer") {   // the asset, if given, is dropped (one currency)
      std::string p1, p2, asset;
      if (!expect("(") || !ident(p1) || !expect(",") || !ident(p2)) return false;
      if (is(",")) { ++p; if (!ident(asset)) return false; }
      if (!expect(")")) return false;
      o = "(payoff ";
      put_te(o, *t0);
      o += " " + p1 + " " + p2 + ")";
      return true;
    }
    if (k == "scale") {
      std::string e, c;
      if (!expect("(") || !expr(t0, e) || !expect(",") || !contract(t0, c) || !expect(")")) return false;
      o = "(mult " + e + " " + c + ")";
      return true;
    }
    if (k == "translate") {
      TP t;
      std::string c;
      if (!expect("(") || !texp(t) || !expect(",") || !contract(tplus(t0, t), c) || !expect(")")) return false;
      o = c;
      return true;
    }
    if (k == "both") {
      std::string a, b;
      if (!expect("(") || !contract(t0, a) || !expect(",") || !contract(t0, b) || !expect(")")) return false;
      o = "(add " + a + " " + b + ")";
      return true;
    }
    if (k == "all") {   // all[c1, ..., cn] = both(c1, both(..., cn))
      std::vector<std::string> cs;
      if (!expect("[")) return false;
      do {
        if (!cs.empty()) ++p;
        std::string c;
        if (!contract(t0, c)) return false;
        cs.push_back(c);
      } while (is(","));
      if (!expect("]")) return false;
      o = cs.back();
      for (size_t i = cs.size() - 1; i-- > 0;) o = "(add " + cs[i] + " " + o + ")";
      return true;
    }
    if (k == "ifWithin") {
      std::string e, a, b;
      TP t;
      if (!expect("(") || !expr(t0, e) || !expect(",") || !texp(t) || !expect(",") || !contract(t0, a) ||
          !expect(",") || !contract(t0, b) || !expect(")"))
        return false;
      o = "(loopif " + e + " " + a + " " + b + " ";
      put_te(o, *t);
      o += ")";
      return true;
    }
    if (k == "if") {   // the condition checked at t0 only: ifWithin with period 0
      std::string e, a, b;
      if (!expect("(") || !expr(t0, e) || !expect(",") || !contract(t0, a) || !expect(",") || !contract(t0, b) ||
          !expect(")"))
        return false;
      o = "(if " + e + " " + a + " " + b + ")";
      return true;
    }
    --p;
    return fail("unknown contract '" + k + "'");
  }

  // --- expressions: tau_e(e, t0), infix operators by precedence
  bool expr(const TP& t0, std::string& o) { return disj(t0, o); }
  bool disj(const TP& t0, std::string& o) {
    if (!conj(t0, o)) return false;
    while (is("||")) {
      ++p;
      std::string r;
      if (!conj(t0, r)) return false;
      o = "(or " + o + " " + r + ")";
    }
    return true;
  }
  bool conj(const TP& t0, std::string& o) {
    if (!cmp(t0, o)) return false;
    while (is("&&")) {
      ++p;
      std::string r;
      if (!cmp(t0, r)) return false;
      o = "(and " + o + " " + r + ")";
    }
    return true;
  }
  bool cmp(const TP& t0, std::string& o) {
    if (!sum(t0, o)) return false;
    if (is("<") || is("<=") || is(">") || is(">=") || is("==")) {
      const std::string op = cur().text;
      ++p;
      std::string r;
      if (!sum(t0, r)) return false;
      if (op == "<") o = "(lt " + o + " " + r + ")";
      else if (op == "<=") o = "(leq " + o + " " + r + ")";
      else if (op == ">") o = "(lt " + r + " " + o + ")";
      else if (op == ">=") o = "(leq " + r + " " + o + ")";
      else o = "(eq " + o + " " + r + ")";
    }
    return true;
  }
  bool sum(const TP& t0, std::string& o) {
    if (!prod(t0, o)) return false;
    while (is("+") || is("-")) {
      const bool add = is("+");
      ++p;
      std::string r;
      if (!prod(t0, r)) return false;
      o = std::string(add ? "(add " : "(sub ") + o + " " + r + ")";
    }
    return true;
  }
  bool prod(const TP& t0, std::string& o) {
    if (!unary(t0, o)) return false;
    while (is("*") || is("/")) {
      const bool mul = is("*");
      ++p;
      std::string r;
      if (!unary(t0, r)) return false;
      o = std::string(mul ? "(mult " : "(div ") + o + " " + r + ")";
    }
    return true;
  }
  bool unary(const TP& t0, std::string& o) {
    const Deeper d(*this);
    if (!d.ok) return fail("expression nested too deeply");
    if (is("-")) {
      ++p;
      std::string x;
      if (!unary(t0, x)) return false;
      o = "(neg " + x + ")";
      return true;
    }
    if (is("!")) {
      ++p;
      std::string x;
      if (!unary(t0, x)) return false;
      o = "(not " + x + ")";
      return true;
    }
    return primary(t0, o);
  }
  bool number(double& v) {
    if (cur().kind != Tok::NUM) return fail("expected a number");
    char* end = nullptr;
    v = std::strtod(cur().text.c_str(), &end);
    if (!end || *end || !std::isfinite(v)) return fail("malformed number '" + cur().text + "'");
    ++p;
    return true;
  }
  bool primary(const TP& t0, std::string& o) {
    const Deeper d(*this);
    if (!d.ok) return fail("expression nested too deeply");
    if (is("(")) {
      ++p;
      return expr(t0, o) && expect(")");
    }
    if (cur().kind == Tok::NUM) {
      double v;
      if (!number(v)) return false;
      char b[64];
      std::snprintf(b, sizeof b, "(real %.17g)", v);
      o = b;
      return true;
    }
    if (cur().kind != Tok::ID) return fail("expected an expression");
    const std::string k = cur().text;
    ++p;
    if (k == "true" || k == "false") {
      o = "(bool " + k + ")";
      return true;
    }
    if (k == "obs") {   // tau_e(obs(l, i), t0) = model(l, t0 + i)
      std::string label;
      if (!expect("(") || !ident(label) || !expect(",")) return false;
      bool negative = false;
      if (is("-")) { negative = true; ++p; }
      int64_t i;
      if (cur().kind != Tok::NUM || !day_numeral(cur().text, i))
        return fail("an observation offset must be an integer of at most 31 bits");
      if (negative) i = -i;
      ++p;
      if (!expect(")")) return false;
      o = "(model " + label + " ";
      put_te(o, *tplus(t0, integer(i)));
      o += ")";
      return true;
    }
    // operators in prefix form: op(e1, ..., en)
    static const struct { const char* name; int arity; } ops[] = {
        {"add", 2}, {"sub", 2}, {"mult", 2}, {"div", 2}, {"min", 2}, {"max", 2}, {"lt", 2}, {"leq", 2},
        {"eq", 2}, {"and", 2}, {"or", 2}, {"neg", 1}, {"not", 1}, {"cond", 3}};
    for (const auto& op : ops) {
      if (k != op.name) continue;
      std::vector<std::string> args;
      if (!expect("(")) return false;
      for (int a = 0; a < op.arity; ++a) {
        if (a > 0 && !expect(",")) return false;
        std::string x;
        if (!expr(t0, x)) return false;
        args.push_back(x);
      }
      if (!expect(")")) return false;
      if (k == "cond") o = "(if " + args[0] + " " + args[1] + " " + args[2] + ")";   // tau_e(cond) = if
      else if (op.arity == 1) o = "(" + k + " " + args[0] + ")";
      else o = "(" + k + " " + args[0] + " " + args[1] + ")";
      return true;
    }
    --p;
    return fail("unknown operator or name '" + k + "'");
  }
};

int cl_to_il(const char* text, size_t len, std::string& il, std::string& err) {
  Lexer lx{text, len};
  if (!lx.run()) { err = lx.err; return PMC_E_PARSE; }
  Compiler cc{lx.toks};
  std::string o;
  if (!cc.contract(nat(0), o)) { err = cc.err; return PMC_E_PARSE; }
  if (cc.cur().kind != Tok::END) { cc.fail("text after the contract"); err = cc.err; return PMC_E_PARSE; }
  il = o;
  return PMC_OK;
}

}  // namespace

extern "C" int pmc_contract_compile(const char* cl_text, size_t len, char* il_out, size_t cap, size_t* il_len) {
  if ((!cl_text && len) || !il_len) return pmc::ctx_fail(nullptr, PMC_E_ARG, "null argument");
  std::string il, err;
  const int st = cl_to_il(cl_text, len, il, err);
  if (st != PMC_OK) return pmc::ctx_fail(nullptr, st, "contract: " + err);
  *il_len = il.size();
  if (il_out && cap) {
    const size_t n = std::min(cap - 1, il.size());
    std::memcpy(il_out, il.data(), n);
    il_out[n] = 0;
  }
  return PMC_OK;
}

extern "C" int pmc_contract_load(pmc_ctx* ctx, const char* cl_text, size_t len, const char* const* asset_labels,
                                 int n_assets, const char* const* param_labels, int n_params,
                                 const char* const* tvar_names, int n_tvars, pmc_payoff** out) {
  if ((!cl_text && len) || !out) return pmc::ctx_fail(ctx, PMC_E_ARG, "null argument");
  std::string il, err;
  const int st = cl_to_il(cl_text, len, il, err);
  if (st != PMC_OK) return pmc::ctx_fail(ctx, st, "contract: " + err);
  return pmc_payoff_load(ctx, il.data(), il.size(), asset_labels, n_assets, param_labels, n_params, tvar_names,
                         n_tvars, out);
}
