"""Contract language CL: syntax, trace semantics, instantiation and the
compiler to the payoff language (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Used to check the payoff-language semantics (Fig. 3 and its readings)
against the paper's soundness theorem: for a compiled contract, the sum of
the discounted trace equals the value of the compiled expression
(Thm. 1(ii), Sec. 4).

Syntax (Fig. 1), as tuples:
  contracts  ('zero',) | ('transfer', p1, p2) | ('scale', e, c)
             | ('translate', T, c) | ('ifwithin', e, T, c1, c2) | ('both', c1, c2)
  expressions ('obs', label, i) | ('lit', float) | ('blit', bool)
             | ('op', name, e1, ..., en)   name in add sub mult div min max lt leq eq and or neg not cond
  templates  ('n', k) | ('v', name)
The asset of a transfer is omitted: compilation drops it (Sec. 4) and the
two-party view of Fig. 3 counts one currency.

Trace semantics (Sec. 2, after Bahr, Berthold and Elsman): a contract at the
current time denotes a trace day -> flow from p1 to p2 (positive) or back
(negative).  transfer flows one unit on day 0; scale multiplies by the
expression evaluated on day 0; translate(t, c) delays c by T[t] days and
evaluates it in the environment advanced by T[t]; both adds; ifWithin(e, t,
c1, c2) takes c1 at the first day i <= T[t] where e holds (delayed by i,
environment advanced by i), else c2 at day T[t].
"""
from __future__ import annotations

from collections import defaultdict

from .il import tsem

OPS = {"add": 2, "sub": 2, "mult": 2, "div": 2, "min": 2, "max": 2, "lt": 2, "leq": 2, "eq": 2,
       "and": 2, "or": 2, "neg": 1, "not": 1, "cond": 3}


# ------------------------------------------------------------ expressions ---
def eval_exp(e, rho, shift):
    """E[e] with observables read at day i + shift."""
    k = e[0]
    if k == "obs":
        return rho(e[1], e[2] + shift)
    if k == "lit":
        return float(e[1])
    if k == "blit":
        return bool(e[1])
    name, args = e[1], [eval_exp(a, rho, shift) for a in e[2:]]
    if name == "cond":
        return args[1] if args[0] else args[2]
    from .il import binop, unop
    if name in ("neg", "not"):
        return unop(name, args[0])
    return binop(name, args[0], args[1])


# -------------------------------------------------------- trace semantics ---
def trace(c, rho, delta, p1="X", p2="Y", shift=0):
    """C[c](rho, delta) as {day: flow p1 -> p2}; ``shift`` is the absolute
    day of the contract's current time."""
    out = defaultdict(float)

    def go(c, start, scale):
        k = c[0]
        if k == "zero":
            return
        if k == "transfer":
            if (c[1], c[2]) == (p1, p2):
                out[start] += scale
            elif (c[1], c[2]) == (p2, p1):
                out[start] -= scale
            return
        if k == "scale":
            go(c[2], start, scale * eval_exp(c[1], rho, start))
            return
        if k == "translate":
            go(c[2], start + tsem(c[1], delta), scale)
            return
        if k == "both":
            go(c[1], start, scale)
            go(c[2], start, scale)
            return
        if k == "ifwithin":
            n = tsem(c[2], delta)
            for i in range(n + 1):
                if eval_exp(c[1], rho, start + i) is True:
                    go(c[3], start + i, scale)
                    return
            go(c[4], start + n, scale)
            return
        raise ValueError(k)

    go(c, shift, 1.0)
    return dict(out)


def horizon(c, delta):
    """A conservative horizon HOR (Sec. 4): the latest day a flow can occur."""
    k = c[0]
    if k in ("zero", "transfer"):
        return 0
    if k == "scale":
        return horizon(c[2], delta)
    if k == "translate":
        return tsem(c[1], delta) + horizon(c[2], delta)
    if k == "both":
        return max(horizon(c[1], delta), horizon(c[2], delta))
    if k == "ifwithin":
        return tsem(c[2], delta) + max(horizon(c[3], delta), horizon(c[4], delta))
    raise ValueError(k)


# ----------------------------------------------------------- instantiation --
def inst(c, delta):
    """Definition 1: replace template variables by their values."""
    k = c[0]
    if k in ("zero", "transfer"):
        return c
    if k == "scale":
        return ("scale", c[1], inst(c[2], delta))
    if k == "translate":
        return ("translate", ("n", tsem(c[1], delta)), inst(c[2], delta))
    if k == "both":
        return ("both", inst(c[1], delta), inst(c[2], delta))
    if k == "ifwithin":
        return ("ifwithin", c[1], ("n", tsem(c[2], delta)), inst(c[3], delta), inst(c[4], delta))
    raise ValueError(k)


def template_closed(c):
    """The TC predicate (Fig. 2)."""
    k = c[0]
    if k in ("zero", "transfer"):
        return True
    if k == "scale":
        return template_closed(c[2])
    if k == "translate":
        return c[1][0] == "n" and template_closed(c[2])
    if k == "both":
        return template_closed(c[1]) and template_closed(c[2])
    if k == "ifwithin":
        return c[2][0] == "n" and template_closed(c[3]) and template_closed(c[4])
    raise ValueError(k)


# ------------------------------------------------------------- compilation --
def tplus_smart(a, b):
    """Smart constructor of Sec. 4: numerals are added, otherwise tplus."""
    if a[0] in ("n", "z") and b[0] in ("n", "z"):
        v = a[1] + b[1]
        return ("n", v) if v >= 0 and a[0] == "n" and b[0] == "n" else ("z", v)
    return ("tplusz", a, b) if "z" in (a[0], b[0]) or a[0] == "tplusz" or b[0] == "tplusz" else ("tplus", a, b)


def compile_exp(e, t0):
    """tau_e(e, t0): observables become model(l, t0 + i)."""
    k = e[0]
    if k == "obs":
        i = e[2]
        return ("model", e[1], tplus_smart(t0, ("n", i) if i >= 0 else ("z", i)))
    if k == "lit":
        return ("real", float(e[1]))
    if k == "blit":
        return ("bool", bool(e[1]))
    name, args = e[1], [compile_exp(a, t0) for a in e[2:]]
    if name == "cond":
        return ("if", args[0], args[1], args[2])
    if name in ("neg", "not"):
        return ("un", name, args[0])
    return ("bin", name, args[0], args[1])


def compile_contract(c, t0=("n", 0)):
    """tau_c(c, t0) (Sec. 4); ifWithin becomes loopif with its own branches
    (the paper prints c_0, c_1 where c_1, c_2 are meant)."""
    k = c[0]
    if k == "zero":
        return ("real", 0.0)
    if k == "transfer":
        return ("payoff", t0, c[1], c[2])
    if k == "scale":
        return ("bin", "mult", compile_exp(c[1], t0), compile_contract(c[2], t0))
    if k == "translate":
        return compile_contract(c[2], tplus_smart(t0, c[1]))
    if k == "both":
        return ("bin", "add", compile_contract(c[1], t0), compile_contract(c[2], t0))
    if k == "ifwithin":
        return ("loopif", compile_exp(c[1], t0), compile_contract(c[3], t0), compile_contract(c[4], t0), c[2])
    raise ValueError(k)


def to_text(e):
    """IL AST -> IL text (the reader's syntax)."""
    k = e[0]

    def t(x):
        if x[0] == "n":
            return str(x[1])
        if x[0] == "z":
            return f"(int {x[1]})"
        if x[0] == "v":
            return f"(tvar {x[1]})"
        if x[0] == "tplus":
            return f"(tplus {t(x[1])} {t(x[2])})"
        return f"(tplusz {t(x[1])} {t(x[2])})"

    if k == "real":
        return f"(real {float(e[1])!r})"
    if k == "bool":
        return f"(bool {'true' if e[1] else 'false'})"
    if k == "nat":
        return f"(nat {e[1]})"
    if k == "now":
        return "(now)"
    if k == "texpr":
        return f"(t {t(e[1])})"
    if k == "model":
        return f"(model {e[1]} {t(e[2])})"
    if k == "payoff":
        return f"(payoff {t(e[1])} {e[2]} {e[3]})"
    if k == "if":
        return f"(if {to_text(e[1])} {to_text(e[2])} {to_text(e[3])})"
    if k == "loopif":
        return f"(loopif {to_text(e[1])} {to_text(e[2])} {to_text(e[3])} {t(e[4])})"
    if k == "un":
        return f"({e[1]} {to_text(e[2])})"
    return f"({e[1]} {to_text(e[2])} {to_text(e[3])})"
