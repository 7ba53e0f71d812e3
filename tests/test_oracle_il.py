"""Pins for the oracle's payoff-language reader, type check, semantics and
grid (CPU only)."""
import itertools
import math

import numpy as np
import pytest

from oracle import grid
from oracle.il import (ILParseError, ILTemplateError, ILTypeError, il_eval, loopif_recursive,
                       parse, template_vars, tsem, typeof)

from golden_io import all_fixtures, load


@pytest.mark.parametrize("path", all_fixtures())
def test_worked_examples(path):
    """Worked examples of the paper (fixtures cite the passage)."""
    rec = load(path)
    e = parse(rec["il"])
    assert typeof(e) == "R"

    def rho(label, day):
        return rec["obs"][(label, day)]

    base = rec["disc"]
    v = il_eval(e, rho, rec["tenv"], 0, 0, lambda k: base ** k, *rec["parties"])
    assert v == pytest.approx(rec["expected"], rel=1e-15, abs=1e-15)


def test_reader_rejects_malformed():
    bad = ["", "(", "(add (real 1.0))", "(real x)", "(model S)", "(payoff -1 X Y)",
           "(foo (real 1.0))", "(real 1.0) (real 2.0)", "(nat -3)", "(loopif (bool true) (real 1.0) (real 2.0))",
           "real", "(model S (int))", "(t (int 3))"]
    for s in bad:
        with pytest.raises(ILParseError):
            parse(s)


def test_type_check():
    ok = {"(add (real 1.0) (real 2.0))": "R", "(lt (now) (t 3))": "B", "(add (nat 1) (t (tvar v)))": "N",
          "(if (bool true) (real 1.0) (real 2.0))": "R", "(not (lt (real 1.0) (real 2.0)))": "B",
          "(eq (bool true) (bool false))": "B", "(min (nat 1) (nat 2))": "N"}
    for s, t in ok.items():
        assert typeof(parse(s)) == t
    bad = ["(add (real 1.0) (nat 1))", "(mult (nat 2) (nat 3))", "(and (real 1.0) (bool true))",
           "(if (real 1.0) (real 1.0) (real 2.0))", "(if (bool true) (real 1.0) (nat 2))",
           "(neg (bool true))", "(not (real 1.0))", "(sub (now) (nat 1))", "(lt (real 1.0) (now))",
           "(loopif (real 0.0) (real 1.0) (real 1.0) 3)"]
    for s in bad:
        with pytest.raises(ILTypeError):
            typeof(parse(s))
    with pytest.raises(ILTypeError):
        typeof(parse("(model Q 0)"), {"S"})


def test_template_semantics():
    d = {"a": 3, "b": 4}
    assert tsem(("tplus", ("v", "a"), ("n", 5)), d) == 8
    assert tsem(("tplusz", ("z", -7), ("v", "b")), d) == -3
    with pytest.raises(ILTemplateError):
        tsem(("v", "zz"), d)
    with pytest.raises(ILTemplateError):
        tsem(("v", "a"), {"a": -1})
    assert template_vars(parse("(loopif (lt (t (tvar x)) (now)) (model S (tvar y)) (real 0.0) (tvar z))")) == {"x", "y", "z"}


def _rand_env(seed, days=range(-5, 40)):
    g = np.random.default_rng(seed)
    tab = {("S", d): float(g.uniform(50, 150)) for d in days}
    return (lambda l, d: tab[(l, d)]), tab


def test_loopif_matches_recursive_definition():
    """The iterative loopif equals the recursion of Fig. 3 (iter n t0')."""
    e = parse("(loopif (lt (real 120.0) (model S 1)) (mult (model S 2) (payoff 1 X Y)) "
              "(sub (model S 0) (payoff 3 X Y)) (tvar n))")
    d = lambda k: 0.97 ** k
    for seed in range(20):
        rho, _ = _rand_env(seed)
        for n in range(0, 8):
            for t0 in (0, 3):
                got = il_eval(e, rho, {"n": n}, t0, 0, d, "X", "Y")
                ref = loopif_recursive(
                    n, t0,
                    lambda s: rho("S", 1 + s) > 120.0,
                    lambda s: rho("S", 2 + s) * d(1 + s),
                    lambda s: rho("S", 0 + s) - d(3 + s))
                assert got == ref


def test_loopif_zero_iterations_is_if():
    rho, _ = _rand_env(1)
    d = lambda k: 0.9 ** k
    a = parse("(loopif (lt (real 100.0) (model S 2)) (model S 3) (payoff 4 X Y) 0)")
    b = parse("(if (lt (real 100.0) (model S 2)) (model S 3) (payoff 4 X Y))")
    for t0 in range(4):
        assert il_eval(a, rho, {}, t0, 0, d, "X", "Y") == il_eval(b, rho, {}, t0, 0, d, "X", "Y")


def test_contract_algebra_special_cases():
    """zero -> 0; scale is multiplication; both is addition; a transfer
    translated by k is d(k); parties swapped negate, unrelated give 0."""
    rho, _ = _rand_env(2)
    d = lambda k: math.exp(-0.01 * k)
    ev = lambda s, p=("X", "Y"): il_eval(parse(s), rho, {"k": 7}, 0, 0, d, *p)
    assert ev("(real 0.0)") == 0.0
    c = "(mult (model S 3) (payoff (tvar k) X Y))"
    assert ev(f"(mult (real 2.5) {c})") == 2.5 * ev(c)
    c2 = "(if (lt (model S 1) (model S 2)) (payoff 2 X Y) (neg (payoff 4 X Y)))"
    assert ev(f"(add {c} {c2})") == ev(c) + ev(c2)
    assert ev("(payoff (tvar k) X Y)") == d(7)
    assert ev("(payoff (tplus (tvar k) 3) X Y)") == d(10)
    assert ev(c, ("Y", "X")) == -ev(c)
    assert ev(c, ("X", "Z")) == 0.0


def test_now_and_texpr_values():
    rho, _ = _rand_env(3)
    e = parse("(loopif (lt (now) (t 0)) (real 1.0) (real 2.0) 10)")
    d = lambda k: 1.0
    # now = 4: condition t0' > 4 first holds at t0' = 5 <= 10
    assert il_eval(e, rho, {}, 0, 4, d, "X", "Y") == 1.0
    assert il_eval(e, rho, {}, 0, 10, d, "X", "Y") == 2.0
    assert il_eval(parse("(t (tplus 2 (tvar a)))"), rho, {"a": 5}, 3, 0, d, "X", "Y") == 10


def test_ieee_division_and_minmax():
    rho, _ = _rand_env(4)
    d = lambda k: 1.0
    ev = lambda s: il_eval(parse(s), rho, {}, 0, 0, d, "X", "Y")
    assert ev("(div (real 1.0) (real 0.0))") == math.inf
    assert math.isnan(ev("(div (real 0.0) (real 0.0))"))
    assert ev("(min (div (real 0.0) (real 0.0)) (real 3.0))") == 3.0
    assert ev("(max (real 3.0) (div (real 0.0) (real 0.0)))") == 3.0


def _days_read_by_evaluation(e, delta, rho):
    seen = set()

    def tracing(label, day):
        seen.add((label, day))
        return rho(label, day)

    il_eval(e, tracing, delta, 0, 0, lambda k: 1.0, "X", "Y")
    return seen


def test_grid_covers_every_read_and_is_tight():
    """Brute force: over many scenarios every day that evaluation reads is in
    the planned set, and scenarios that never trigger the loop condition
    read exactly the planned set."""
    e = parse("(add (loopif (lt (real 130.0) (model S 2)) (model S 3) (model S (int -2)) (tvar n)) "
              "(loopif (lt (model S 0) (real 0.0)) (real 0.0) (model S (tplus (tvar m) 1)) 2))")
    delta = {"n": 4, "m": 3}
    md, pd = grid.reads(e, delta)
    planned = {("S", x) for x in md["S"]}
    for seed in range(60):
        rho, _ = _rand_env(seed)
        assert _days_read_by_evaluation(e, delta, rho) <= planned
    # with no condition ever true, only the first loop's first branch (days
    # 3+0 .. 3+4; all but day 7 are read elsewhere) is never evaluated
    never = lambda l, d: 100.0
    assert _days_read_by_evaluation(e, delta, never) == planned - {("S", 7)}
    assert grid.slots(e, delta, ["S"]) == sorted(x for x in md["S"] if x > 0)
    assert grid.horizon(e, delta) == max(md["S"])


def test_grid_of_configs():
    import workloads as W
    c2 = parse(W.WORST_OF_AUTOCALL)
    assert grid.slots(c2, {"N": 4}, ["S1", "S2", "S3"]) == [1, 2, 3, 4, 5]
    assert grid.slots(c2, {"N": 0}, ["S1", "S2", "S3"]) == [1]
    c3 = parse(W.DOWN_AND_OUT_CALL)
    assert grid.slots(c3, {"T": 1260}, ["S"]) == list(range(1, 1261))
    md, pd = grid.reads(c3, {"T": 1260})
    assert pd == {1260} and min(md["S"]) == 0
    c1 = parse(W.EUROPEAN_CALL)
    assert grid.slots(c1, {"T": 252}, ["S"]) == [252]
