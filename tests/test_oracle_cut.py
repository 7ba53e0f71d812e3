"""Pins for the time-parameterised payoffs of Sec. 4.1 (CPU only)."""
import math

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


# ---- pricing at a current day on a price history (Sec. 4.1) ---------------
def _prob(cfg, **over):
    from oracle.mc import Problem
    kw = dict(asset_labels=cfg.asset_labels, param_labels=cfg.param_labels, params=cfg.params,
              tenv=cfg.tenv_dict(), spot=cfg.spot, vol=cfg.vol, corr=cfg.corr, rate=cfg.rate,
              years_per_day=cfg.years_per_day, rng=cfg.rng, seed=cfg.seed, precision=cfg.precision)
    il = over.pop("il", cfg.il)
    kw.update(over)
    return Problem(il, **kw)


def test_history_ending_on_day_zero_is_plain_pricing():
    """A history of the spot alone, ending on day 0, is the environment the
    pricing without a history assumes: identical payoffs path by path."""
    import dataclasses
    for cfg in (W.C1, dataclasses.replace(W.C3, tenv=[40]), W.C2):
        ids = np.arange(64)
        plain = _prob(cfg).payoffs(ids)
        hist = _prob(cfg, history=[[s] for s in cfg.spot]).payoffs(ids)
        assert np.array_equal(plain, hist), cfg.name


def test_history_european_is_black_scholes_from_the_current_day():
    """European call (strike 100, 252 days) priced on day 100 of its life on
    a history ending at S = 110: the simulation starts from that price, so
    the price is d(100) times the Black-Scholes call on spot 110 over the
    remaining 152 days (closed form; within 3 standard errors)."""
    from oracle.closed_form import bs_call
    from oracle.mc import estimate
    cfg = W.C1
    n, now = 1 << 14, 100
    hist = [[95.0, 104.0, 110.0]]              # days 98, 99, 100
    prob = _prob(cfg, t_now=now, history=hist)
    assert prob.days == [252]
    p, se = estimate(prob.payoffs(np.arange(n)))
    ypd = cfg.years_per_day
    ref = math.exp(-cfg.rate * now * ypd) * bs_call(110.0, 100.0, cfg.rate, 0.2, (252 - now) * ypd)
    assert abs(p - ref) <= 3 * se, (p, ref, se)


def test_history_commutes_with_contract_reduction():
    """Thm. 4 for n steps: evaluating the cut payoff at current day n on an
    environment whose days up to n are history equals evaluating the
    contract reduced by n days at day 0 with the environment and the
    discount shifted by n.  For a down-and-out whose history (days 0..n)
    stays above the barrier, the reduced contract is the same one with
    T - n days, spot S(n), and d/n = d(n) d: equal path by path on the same
    random stream.  A history that touches the barrier knocks every path
    out: exactly 0."""
    import dataclasses
    cfg = dataclasses.replace(W.C3, tenv=[60])
    T, now = 60, 20
    walk = 100.0 * np.exp(0.01 * np.cumsum(np.random.default_rng(5).normal(size=now + 1)))
    assert walk.min() > 70.0
    ids = np.arange(128)
    e = parse(cfg.il)
    a = _prob(cfg, il=cut_payoff(e), t_now=now, history=[walk]).payoffs(ids)
    b = _prob(dataclasses.replace(cfg, tenv=[T - now], spot=[float(walk[-1])])).payoffs(ids)
    scale = math.exp(-cfg.rate * now * cfg.years_per_day)
    assert np.count_nonzero(a) > 10
    np.testing.assert_allclose(a, scale * b, rtol=1e-12, atol=1e-12)
    # the plain payoff too: every flow of this contract is on day T >= n
    a2 = _prob(cfg, t_now=now, history=[walk]).payoffs(ids)
    np.testing.assert_allclose(a2, a, rtol=0, atol=0)
    hit = walk.copy()
    hit[7] = 69.0
    assert np.all(_prob(cfg, il=cut_payoff(e), t_now=now, history=[hit]).payoffs(ids) == 0.0)


def test_history_days_before_its_first_read_its_first_price():
    """The worst-of autocall reads days 1 - 3 .. 5 (its maturity branch
    looks back three dates from the last shift); on day 2 with a history of
    days 1 and 2 only, the days before read the day-1 prices, and the
    simulated grid is days 3..5."""
    cfg = W.C2
    hist = [[101.0, 99.0], [100.5, 98.0], [102.0, 97.5]]
    prob = _prob(cfg, t_now=2, history=hist)
    assert prob.days == [3, 4, 5]
    rho = prob.env(np.zeros((3, 3)))
    assert rho("S2", -2) == 100.5 and rho("S2", 1) == 100.5 and rho("S2", 2) == 98.0
    assert rho("S3", 0) == 102.0
