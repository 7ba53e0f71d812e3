"""Pins for the time-parameterised payoffs of Sec. 4.1 (CPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle import grid
from oracle.il import cashflows, cut_payoff, il_eval, parse

from golden_io import load, all_fixtures


def _env(seed, labels=("S", "S1", "S2", "S3", "AAPL", "K", "B"), days=range(-5, 1300)):
    g = np.random.default_rng(seed)
    tab = {}
    for l in labels:
        s = 100.0
        for d in days:
            s *= float(np.exp(0.02 * g.normal()))
            tab[(l, d)] = s
    return lambda l, d: tab[(l, d)]


CASES = [
    (W.EUROPEAN_CALL, {"T": 40}, {"K": 100.0}),
    (W.DOWN_AND_OUT_CALL, {"T": 60}, {"K": 100.0, "B": 80.0}),
    (W.WORST_OF_AUTOCALL, {"N": 4}, {}),
    ("(add (mult (real 100.0) (payoff (tvar t0) X Y)) (loopif (lt (real 104.0) (model S 1)) "
     "(mult (model S 1) (payoff 1 X Y)) (neg (payoff 3 Y X)) (tvar t1)))", {"t0": 10, "t1": 30}, {}),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_cut_soundness_n_steps(case):
    """Thm. 5: the cut expression evaluated at current time n equals the sum
    of the discounted cashflows at days >= n (here: of the same payoff
    expression, whose per-day cashflows are extracted by evaluating it with
    an indicator discount function)."""
    il, delta, params = CASES[case]
    e = parse(il)
    cut = cut_payoff(e)
    H = grid.horizon(e, delta)
    d = lambda day: 0.999 ** day
    for seed in range(6):
        base = _env(seed)
        rho = lambda l, day: params[l] if l in params else base(l, day)
        flows = cashflows(e, rho, delta, 0, "X", "Y", H)
        full = il_eval(e, rho, delta, 0, 0, d, "X", "Y")
        assert full == pytest.approx(sum(d(k) * f for k, f in enumerate(flows)), rel=1e-12, abs=1e-12)
        for n in (0, 1, 2, 5, H // 2, H, H + 1):
            got = il_eval(cut, rho, delta, 0, n, d, "X", "Y")
            ref = sum(d(k) * f for k, f in enumerate(flows) if k >= n)
            assert got == pytest.approx(ref, rel=1e-12, abs=1e-12), (n, got, ref)


def test_cut_at_time_zero_is_identity():
    for il, delta, params in CASES:
        e = parse(il)
        for seed in range(3):
            base = _env(seed)
            rho = lambda l, day: params[l] if l in params else base(l, day)
            assert il_eval(cut_payoff(e), rho, delta, 0, 0, lambda k: 0.97 ** k, "X", "Y") == \
                il_eval(e, rho, delta, 0, 0, lambda k: 0.97 ** k, "X", "Y")


def test_example4_structure():
    """Example 4 (Sec. 4.1): cutting Example 3 guards each payoff with its own
    day against now, and leaves the rest unchanged."""
    rec = load(all_fixtures("example3")[0])
    e = parse(rec["il"])
    c = cut_payoff(e)
    # first summand: 100 * if(t0 < now, 0, payoff(t0))
    first = c[2]
    assert first[0] == "bin" and first[1] == "mult"
    guard = first[3]
    assert guard[0] == "if" and guard[1] == ("bin", "lt", ("texpr", ("v", "t0")), ("now",))
    assert guard[2] == ("real", 0.0) and guard[3] == e[2][3]
    rho = lambda l, d: rec["obs"][(l, d)]
    dd = lambda k: 0.99 ** k
    # now = 15: only the day-30 leg remains; now = 31: nothing remains
    assert il_eval(c, rho, rec["tenv"], 0, 15, dd, "you", "me") == pytest.approx(20 * 0.99 ** 30)
    assert il_eval(c, rho, rec["tenv"], 0, 31, dd, "you", "me") == 0.0
