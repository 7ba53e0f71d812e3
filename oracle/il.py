"""Payoff intermediate language: syntax, type check and semantics (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Syntax follows the IL grammar of Sec. 3 and the Coq types of Sec. 5
(``ILExpr`` with constructors ILIf, ILFloat, ILNat, ILBool, ILtexpr, ILNow,
ILModel, ILUnExpr, ILBinExpr, ILLoopIf, ILPayoff; template expressions
``ILTExpr`` = n | v | tplus and ``ILTExprZ`` which adds integer literals and
their addition).  The semantics is Fig. 3, with the readings listed below.

Concrete text syntax (S-expressions, one node per parenthesised form)::

    e  ::= (now) | (real F) | (nat N) | (bool true|false) | (t T)
         | (model LABEL Z) | (payoff T P1 P2)
         | (if e e e) | (loopif e e e T)
         | (neg e) | (not e) | (OP e e)
    OP ::= add | sub | mult | div | min | max | lt | leq | eq | and | or
    T  ::= N | (tvar NAME) | (tplus T T)
    Z  ::= T | (int I) | (tplusz Z Z)

AST nodes are tuples: ('now',), ('real', f), ('nat', n), ('bool', b),
('texpr', T), ('model', label, Z), ('payoff', T, p1, p2),
('if', c, a, b), ('loopif', c, a, b, T), ('un', op, e), ('bin', op, x, y).
Template nodes: ('n', k), ('v', name), ('tplus', T, T), ('z', i),
('tplusz', Z, Z).

Readings of the paper taken here (each is also listed in the design notes):

* payoff discounting (Fig. 3): the discount is taken at the template value
  plus the current loop shift t0, i.e. d(T[t]delta + t0).  The Futhark
  backend's ``disc[t0]`` and Thm. 1(ii) (a transfer inside ifWithin is
  discounted on the day it fires) both require the shift.
* loopif (Fig. 3): iter(n, t0') checks the condition at t0'; true gives the
  first branch at t0'; false with n = 0 gives the second branch at t0';
  false with n > 0 continues with iter(n-1, t0'+1).  Evaluation starts with
  iter(T[t]delta, t0), so the condition is tested on the n+1 days
  t0 .. t0+n.  This is the recursion of the Haskell ``loopif`` in Sec. 6.1.
* operators: the grammar's operator list is open; this build fixes
  add, sub, mult, div, min, max, lt, leq, eq, and, or, neg, not.  ``and`` and
  ``or`` are not short-circuiting (IL is pure).  Division follows IEEE 754.
  min/max return the other operand when one is NaN (IEEE minNum/maxNum).
* value types (Fig. 3 domain N + R + B): N values come from ``now``, ``nat``
  and ``t``; N may be added, min/max-ed and compared with N; R and N are not
  mixed.  Observables are real-valued.
"""
from __future__ import annotations

import math

import numpy as np

BINOPS = ("add", "sub", "mult", "div", "min", "max", "lt", "leq", "eq", "and", "or")
UNOPS = ("neg", "not")


class ILParseError(ValueError):
    pass


class ILTypeError(ValueError):
    pass


class ILTemplateError(ValueError):
    pass


# ----------------------------------------------------------------------------
# Reader
# ----------------------------------------------------------------------------
def _tokens(text: str):
    out = []
    for line in text.splitlines():
        line = line.split(";", 1)[0]
        out.extend(line.replace("(", " ( ").replace(")", " ) ").split())
    return out


def _read(tokens, pos):
    if pos >= len(tokens):
        raise ILParseError("unexpected end of input")
    tok = tokens[pos]
    if tok == ")":
        raise ILParseError("unexpected ')'")
    if tok != "(":
        return tok, pos + 1
    items = []
    pos += 1
    while True:
        if pos >= len(tokens):
            raise ILParseError("missing ')'")
        if tokens[pos] == ")":
            return items, pos + 1
        item, pos = _read(tokens, pos)
        items.append(item)


def _int_atom(x, what):
    if not isinstance(x, str):
        raise ILParseError(f"{what}: expected an integer, got a list")
    try:
        return int(x, 10)
    except ValueError:
        raise ILParseError(f"{what}: bad integer {x!r}") from None


def _texpr(s):
    """ILTExpr: n | (tvar v) | (tplus T T)."""
    if isinstance(s, str):
        k = _int_atom(s, "template numeral")
        if k < 0:
            raise ILParseError("template numeral must be a natural number")
        return ("n", k)
    if len(s) == 2 and s[0] == "tvar" and isinstance(s[1], str):
        return ("v", s[1])
    if len(s) == 3 and s[0] == "tplus":
        return ("tplus", _texpr(s[1]), _texpr(s[2]))
    raise ILParseError(f"bad template expression {s!r}")


def _texprz(s):
    """ILTExprZ: T | (int i) | (tplusz Z Z)."""
    if isinstance(s, list) and len(s) == 2 and s[0] == "int":
        return ("z", _int_atom(s[1], "int literal"))
    if isinstance(s, list) and len(s) == 3 and s[0] == "tplusz":
        return ("tplusz", _texprz(s[1]), _texprz(s[2]))
    return _texpr(s)


def _expr(s):
    if isinstance(s, str):
        raise ILParseError(f"bare atom {s!r} where an expression is expected")
    if not s:
        raise ILParseError("empty form")
    head = s[0]
    if not isinstance(head, str):
        raise ILParseError("form head must be a symbol")
    n = len(s)
    if head == "now" and n == 1:
        return ("now",)
    if head == "real" and n == 2 and isinstance(s[1], str):
        try:
            return ("real", float(s[1]))
        except ValueError:
            raise ILParseError(f"bad real literal {s[1]!r}") from None
    if head == "nat" and n == 2:
        k = _int_atom(s[1], "nat literal")
        if k < 0:
            raise ILParseError("nat literal must be >= 0")
        return ("nat", k)
    if head == "bool" and n == 2 and s[1] in ("true", "false"):
        return ("bool", s[1] == "true")
    if head == "t" and n == 2:
        return ("texpr", _texpr(s[1]))
    if head == "model" and n == 3 and isinstance(s[1], str):
        return ("model", s[1], _texprz(s[2]))
    if head == "payoff" and n == 4 and isinstance(s[2], str) and isinstance(s[3], str):
        return ("payoff", _texpr(s[1]), s[2], s[3])
    if head == "if" and n == 4:
        return ("if", _expr(s[1]), _expr(s[2]), _expr(s[3]))
    if head == "loopif" and n == 5:
        return ("loopif", _expr(s[1]), _expr(s[2]), _expr(s[3]), _texpr(s[4]))
    if head in UNOPS and n == 2:
        return ("un", head, _expr(s[1]))
    if head in BINOPS and n == 3:
        return ("bin", head, _expr(s[1]), _expr(s[2]))
    raise ILParseError(f"unknown or malformed form {head!r} with {n - 1} arguments")


def parse(text: str):
    """Parse IL text into an AST (raises ILParseError)."""
    toks = _tokens(text)
    sexp, pos = _read(toks, 0)
    if pos != len(toks):
        raise ILParseError("trailing input after expression")
    return _expr(sexp)


# ----------------------------------------------------------------------------
# Type check (value domain N + R + B of Fig. 3)
# ----------------------------------------------------------------------------
def typeof(e, labels=None) -> str:
    """Return 'N', 'R' or 'B' for a well-typed node, else raise ILTypeError.

    ``labels`` (optional) is the set of observable labels the model knows;
    a ``model`` node naming another label is a type error.
    """
    k = e[0]
    if k in ("now", "nat", "texpr"):
        return "N"
    if k == "real":
        return "R"
    if k == "bool":
        return "B"
    if k == "model":
        if labels is not None and e[1] not in labels:
            raise ILTypeError(f"unknown observable {e[1]!r}")
        return "R"
    if k == "payoff":
        return "R"
    if k == "un":
        t = typeof(e[2], labels)
        if e[1] == "neg" and t == "R":
            return "R"
        if e[1] == "not" and t == "B":
            return "B"
        raise ILTypeError(f"{e[1]} applied to {t}")
    if k == "bin":
        op = e[1]
        a, b = typeof(e[2], labels), typeof(e[3], labels)
        if a != b:
            raise ILTypeError(f"{op} applied to {a} and {b}")
        if op in ("add", "min", "max") and a in ("R", "N"):
            return a
        if op in ("sub", "mult", "div") and a == "R":
            return "R"
        if op in ("lt", "leq") and a in ("R", "N"):
            return "B"
        if op == "eq":
            return "B"
        if op in ("and", "or") and a == "B":
            return "B"
        raise ILTypeError(f"{op} applied to {a} and {b}")
    if k in ("if", "loopif"):
        if typeof(e[1], labels) != "B":
            raise ILTypeError(f"{k} condition is not boolean")
        a, b = typeof(e[2], labels), typeof(e[3], labels)
        if a != b:
            raise ILTypeError(f"{k} branches have types {a} and {b}")
        return a
    raise ILTypeError(f"unknown node {k!r}")


# ----------------------------------------------------------------------------
# Template semantics: T[n]delta = n, T[v]delta = delta(v), tplus is +.
# ----------------------------------------------------------------------------
def tsem(t, delta) -> int:
    k = t[0]
    if k in ("n", "z"):
        return t[1]
    if k == "v":
        if t[1] not in delta:
            raise ILTemplateError(f"template variable {t[1]!r} is not bound")
        v = delta[t[1]]
        if not isinstance(v, (int, np.integer)) or v < 0:
            raise ILTemplateError(f"template variable {t[1]!r} must be a natural number")
        return int(v)
    if k in ("tplus", "tplusz"):
        return tsem(t[1], delta) + tsem(t[2], delta)
    raise ILTemplateError(f"bad template node {k!r}")


def template_vars(e, acc=None):
    """Set of template variable names an expression mentions."""
    acc = set() if acc is None else acc

    def tv(t):
        if t[0] == "v":
            acc.add(t[1])
        elif t[0] in ("tplus", "tplusz"):
            tv(t[1])
            tv(t[2])

    def walk(x):
        k = x[0]
        if k == "texpr":
            tv(x[1])
        elif k == "model":
            tv(x[2])
        elif k == "payoff":
            tv(x[1])
        elif k == "loopif":
            walk(x[1]); walk(x[2]); walk(x[3]); tv(x[4])
        elif k == "if":
            walk(x[1]); walk(x[2]); walk(x[3])
        elif k == "un":
            walk(x[2])
        elif k == "bin":
            walk(x[2]); walk(x[3])

    walk(e)
    return acc


# ----------------------------------------------------------------------------
# Operator semantics
# ----------------------------------------------------------------------------
def _fmin(x, y):
    if isinstance(x, float) and math.isnan(x):
        return y
    if isinstance(y, float) and math.isnan(y):
        return x
    return x if x <= y else y


def _fmax(x, y):
    if isinstance(x, float) and math.isnan(x):
        return y
    if isinstance(y, float) and math.isnan(y):
        return x
    return x if x >= y else y


def _div(x, y):
    with np.errstate(all="ignore"):
        return float(np.float64(x) / np.float64(y))


def binop(op, x, y):
    if op == "add":
        return x + y
    if op == "sub":
        return x - y
    if op == "mult":
        return x * y
    if op == "div":
        return _div(x, y)
    if op == "min":
        return _fmin(x, y)
    if op == "max":
        return _fmax(x, y)
    if op == "lt":
        return x < y
    if op == "leq":
        return x <= y
    if op == "eq":
        return x == y
    if op == "and":
        return bool(x) and bool(y)
    if op == "or":
        return bool(x) or bool(y)
    raise ValueError(op)


def unop(op, x):
    if op == "neg":
        return -x
    if op == "not":
        return not x
    raise ValueError(op)


# ----------------------------------------------------------------------------
# Semantics, Fig. 3:  IL[il](rho, delta, t0, t, d, p1, p2)
# ----------------------------------------------------------------------------
def il_eval(e, rho, delta, t0, t, d, p1, p2):
    """Evaluate one payoff expression on one scenario.

    rho(label, day) -> float   external environment (an observable on a day)
    delta                      template environment, name -> natural number
    t0                         accumulated loop shift (natural number)
    t                          current time ``now`` (natural number)
    d(day) -> float            discount function
    p1, p2                     the two parties; flows p1 -> p2 count positive
    """
    k = e[0]
    if k == "texpr":                     # T[t]delta + t0
        return tsem(e[1], delta) + t0
    if k == "real":
        return float(e[1])
    if k == "nat":
        return int(e[1])
    if k == "bool":
        return bool(e[1])
    if k == "un":
        return unop(e[1], il_eval(e[2], rho, delta, t0, t, d, p1, p2))
    if k == "bin":
        return binop(e[1], il_eval(e[2], rho, delta, t0, t, d, p1, p2),
                     il_eval(e[3], rho, delta, t0, t, d, p1, p2))
    if k == "model":                     # rho(l, T[t]delta + t0)
        return rho(e[1], tsem(e[2], delta) + t0)
    if k == "now":
        return t
    if k == "if":
        c = il_eval(e[1], rho, delta, t0, t, d, p1, p2)
        if c is True:
            return il_eval(e[2], rho, delta, t0, t, d, p1, p2)
        return il_eval(e[3], rho, delta, t0, t, d, p1, p2)
    if k == "payoff":                    # +-d(T[t]delta + t0) for matching parties
        q1, q2 = e[2], e[3]
        day = tsem(e[1], delta) + t0
        if q1 == p1 and q2 == p2:
            return d(day)
        if q1 == p2 and q2 == p1:
            return -d(day)
        return 0.0
    if k == "loopif":
        c, a, b = e[1], e[2], e[3]
        # iter(n, t0') of Fig. 3, run as a loop so that long date ranges do
        # not hit Python's recursion limit (``loopif_recursive`` below is the
        # recursion itself; the tests check that both agree)
        n, t0p = tsem(e[4], delta), t0
        while True:
            if il_eval(c, rho, delta, t0p, t, d, p1, p2) is True:
                return il_eval(a, rho, delta, t0p, t, d, p1, p2)
            if n == 0:
                return il_eval(b, rho, delta, t0p, t, d, p1, p2)
            n, t0p = n - 1, t0p + 1
    raise ValueError(f"unknown node {k!r}")


def loopif_recursive(n, t0, cond, e1, e2):
    """The loopif of Fig. 3 written as the recursion itself (used by tests to
    pin the iterative form in ``il_eval``): cond, e1, e2 are functions of the
    shift t0'."""
    if cond(t0):
        return e1(t0)
    if n == 0:
        return e2(t0)
    return loopif_recursive(n - 1, t0 + 1, cond, e1, e2)


def parties(e, acc=None):
    """Set of party names that payoff nodes mention."""
    acc = set() if acc is None else acc
    k = e[0]
    if k == "payoff":
        acc.add(e[2]); acc.add(e[3])
    elif k in ("if", "loopif"):
        parties(e[1], acc); parties(e[2], acc); parties(e[3], acc)
    elif k == "un":
        parties(e[2], acc)
    elif k == "bin":
        parties(e[2], acc); parties(e[3], acc)
    return acc


# ----------------------------------------------------------------------------
# cutPayoff (Sec. 4.1): guard every payoff with "if (t < now) then 0".
# ----------------------------------------------------------------------------
def cut_payoff(e):
    """cutPayoff of Sec. 4.1.  The paper lists the cases for now, model,
    unary and binary operators, if and payoff; this reading recurses through
    every constructor (loopif included) and leaves literals and template
    values unchanged.  A payoff(t, p, q) becomes
    if(lt(t(t), now), 0.0, payoff(t, p, q)): the guard compares the payoff's
    day T[t]delta + t0 with the current time."""
    k = e[0]
    if k == "payoff":
        return ("if", ("bin", "lt", ("texpr", e[1]), ("now",)), ("real", 0.0), e)
    if k in ("if", "loopif"):
        return (k, cut_payoff(e[1]), cut_payoff(e[2]), cut_payoff(e[3])) + tuple(e[4:])
    if k == "un":
        return ("un", e[1], cut_payoff(e[2]))
    if k == "bin":
        return ("bin", e[1], cut_payoff(e[2]), cut_payoff(e[3]))
    return e


def cashflows(e, rho, delta, t, p1, p2, horizon):
    """Per-day discounted-cashflow weights of a payoff expression that is
    linear in its payoff nodes (as compiled contracts are, Sec. 4): the value
    with the discount function replaced by the indicator of day k, for
    k = 0 .. horizon."""
    return [float(il_eval(e, rho, delta, 0, t, lambda day, k=k: 1.0 if day == k else 0.0, p1, p2))
            for k in range(horizon + 1)]
