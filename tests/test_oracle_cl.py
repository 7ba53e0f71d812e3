"""The payoff-language semantics (Fig. 3 with this build's readings) against
the contract language it is compiled from (CPU only): Thm. 1(ii) soundness,
Lemma 2 instantiation soundness, the TC predicate, Example 3, and the
compiled text accepted by the library's loader with the same simulated grid."""
import math

import numpy as np
import pytest

from oracle import cl, grid
from oracle.il import il_eval, parse, typeof


def rand_exp(g, depth, ty):
    if ty == "R":
        k = g.integers(0, 7) if depth > 0 else g.integers(0, 2)
        if k == 0:
            return ("lit", float(np.round(g.uniform(-2, 120), 2)))
        if k == 1:
            return ("obs", "S", int(g.integers(-3, 6)))
        if k in (2, 3, 4):
            op = ["add", "sub", "mult", "min", "max"][g.integers(0, 5)]
            return ("op", op, rand_exp(g, depth - 1, "R"), rand_exp(g, depth - 1, "R"))
        if k == 5:
            return ("op", "cond", rand_exp(g, depth - 1, "B"), rand_exp(g, depth - 1, "R"), rand_exp(g, depth - 1, "R"))
        return ("op", "neg", rand_exp(g, depth - 1, "R"))
    k = g.integers(0, 4) if depth > 0 else 0
    if k == 0:
        return ("op", ["lt", "leq"][g.integers(0, 2)], rand_exp(g, depth - 1, "R"), rand_exp(g, depth - 1, "R"))
    if k == 1:
        return ("op", ["and", "or"][g.integers(0, 2)], rand_exp(g, depth - 1, "B"), rand_exp(g, depth - 1, "B"))
    if k == 2:
        return ("op", "not", rand_exp(g, depth - 1, "B"))
    return ("blit", bool(g.integers(0, 2)))


def rand_tmpl(g):
    return ("v", ["a", "b"][g.integers(0, 2)]) if g.integers(0, 2) else ("n", int(g.integers(0, 6)))


def rand_contract(g, depth):
    k = g.integers(0, 6) if depth > 0 else g.integers(0, 2)
    if k == 0:
        return ("zero",)
    if k == 1:
        return ("transfer",) + [("X", "Y"), ("Y", "X"), ("X", "Z")][g.integers(0, 3)]
    if k == 2:
        return ("scale", rand_exp(g, 2, "R"), rand_contract(g, depth - 1))
    if k == 3:
        return ("translate", rand_tmpl(g), rand_contract(g, depth - 1))
    if k == 4:
        return ("both", rand_contract(g, depth - 1), rand_contract(g, depth - 1))
    return ("ifwithin", rand_exp(g, 2, "B"), rand_tmpl(g), rand_contract(g, depth - 1), rand_contract(g, depth - 1))


def rand_env(g, lo=-12, hi=120):
    tab = {("S", d): float(g.lognormal(np.log(100), 0.2)) for d in range(lo, hi)}
    return lambda l, d: tab[(l, d)]


@pytest.mark.parametrize("seed", range(200))
def test_soundness_theorem_1(seed):
    """Thm. 1(ii): sum_t d(t) tr(t)(p1,p2) equals the compiled expression's
    value at t0 = 0, t = 0; and the compiled expression is real-typed (Thm. 2)."""
    g = np.random.default_rng(seed)
    c = rand_contract(g, 4)
    delta = {"a": int(g.integers(0, 6)), "b": int(g.integers(0, 6))}
    rho = rand_env(g)
    d = lambda day: math.exp(-0.01 * day)
    tr = cl.trace(c, rho, delta)
    lhs = math.fsum(d(t) * v for t, v in tr.items())
    il = cl.compile_contract(c)
    assert typeof(il) == "R"
    rhs = il_eval(il, rho, delta, 0, 0, d, "X", "Y")
    assert rhs == pytest.approx(lhs, rel=1e-12, abs=1e-9)
    assert all(t <= cl.horizon(c, delta) for t in tr)
    # the text form reads back to the same tree
    assert parse(cl.to_text(il)) == il


@pytest.mark.parametrize("seed", range(60))
def test_instantiation_soundness_lemma_2(seed):
    g = np.random.default_rng(1000 + seed)
    c = rand_contract(g, 4)
    delta = {"a": int(g.integers(0, 6)), "b": int(g.integers(0, 6))}
    rho = rand_env(g)
    ci = cl.inst(c, delta)
    assert cl.template_closed(ci)                       # Lemma 1
    assert cl.trace(c, rho, delta) == cl.trace(ci, rho, {"a": 99, "b": 98})


def test_example3_compiles_to_the_printed_expression():
    """Example 3 (Sec. 4): the compiled form is
    100 * payoff(t0) + if(model(AAPL, t0+t1) > 100, (model - 100) * payoff(t0+t1), 0)."""
    obs = ("obs", "AAPL", 0)
    c = ("translate", ("v", "t0"),
         ("both", ("scale", ("lit", 100.0), ("transfer", "you", "me")),
          ("translate", ("v", "t1"),
           ("scale", ("op", "cond", ("op", "lt", ("lit", 100.0), obs), ("op", "sub", obs, ("lit", 100.0)),
                      ("lit", 0.0)), ("transfer", "you", "me")))))
    il = cl.compile_contract(c)
    rho = lambda l, day: {30: 120.0, 10: 90.0}.get(day, 50.0)
    d = lambda k: 0.99 ** k
    v = il_eval(il, rho, {"t0": 10, "t1": 20}, 0, 0, d, "you", "me")
    assert v == pytest.approx(100 * 0.99 ** 10 + 20 * 0.99 ** 30, rel=1e-14)


def test_workload_expressions_match_their_contracts():
    """The hand-written IL of the down-and-out call equals the compiled CL
    contract ifWithin(S <= B, T, zero, if(S > K, scale(S - K, transfer)))
    on random scenarios (parameters as constant observables)."""
    import workloads as W
    S = ("obs", "S", 0)
    K, B = ("obs", "K", 0), ("obs", "B", 0)
    c = ("ifwithin", ("op", "leq", S, B), ("v", "T"), ("zero",),
         ("scale", ("op", "cond", ("op", "lt", K, S), ("op", "sub", S, K), ("lit", 0.0)), ("transfer", "X", "Y")))
    il = cl.compile_contract(c)
    hand = parse(W.DOWN_AND_OUT_CALL)
    for seed in range(20):
        g = np.random.default_rng(seed)
        base = rand_env(g, 0, 60)
        rho = lambda l, d: {"K": 100.0, "B": 85.0}.get(l) or base("S", d)
        dd = lambda k: 0.999 ** k
        for T in (0, 5, 30):
            a = il_eval(il, rho, {"T": T}, 0, 0, dd, "X", "Y")
            b = il_eval(hand, rho, {"T": T}, 0, 0, dd, "X", "Y")
            assert a == pytest.approx(b, rel=1e-14, abs=1e-14)


@pytest.mark.parametrize("seed", range(40))
def test_library_loader_accepts_compiled_contracts_and_plans_the_same_grid(seed):
    """Independent grid planners: the library's (C++) and the oracle's agree
    on the simulated days and the horizon of compiled random contracts."""
    import paper_2108_03076_amd as P
    g = np.random.default_rng(5000 + seed)
    c = rand_contract(g, 4)
    il = cl.compile_contract(c)
    delta = {"a": int(g.integers(0, 6)), "b": int(g.integers(0, 6))}
    pay = P.load_payoff(cl.to_text(il), ["S"], [], ["a", "b"])
    days, hz = pay.grid([delta["a"], delta["b"]])
    assert days == grid.slots(il, delta, ["S"])
    assert hz == grid.horizon(il, delta)
