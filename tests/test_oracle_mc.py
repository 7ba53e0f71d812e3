"""Pins for the oracle's paths and Monte Carlo estimator (CPU only):
closed forms, exact special cases, invariants and brute force."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import mc
from oracle.model import NotPositiveDefinite, cholesky, gbm_paths


def problem(cfg, **over):
    kw = dict(asset_labels=cfg.asset_labels, param_labels=cfg.param_labels, params=cfg.params,
              tenv=cfg.tenv_dict(), spot=cfg.spot, vol=cfg.vol, corr=cfg.corr, rate=cfg.rate,
              years_per_day=cfg.years_per_day, rng=cfg.rng, seed=cfg.seed, precision=cfg.precision)
    il = over.pop("il", cfg.il)
    kw.update(over)
    return mc.Problem(il, **kw)


def test_cholesky_pins():
    c = np.array(W.corr_equi(3, 0.5))
    L = cholesky(c)
    assert np.allclose(L, np.linalg.cholesky(c), rtol=0, atol=1e-15)
    assert np.allclose(L @ L.T, c, rtol=0, atol=1e-15)
    assert np.allclose(L, [[1, 0, 0], [0.5, math.sqrt(3) / 2, 0], [0.5, 0.5 / math.sqrt(3), math.sqrt(2 / 3)]],
                       atol=1e-15)
    g = np.random.default_rng(0)
    for n in (1, 2, 4):
        a = g.normal(size=(n, n))
        spd = a @ a.T + n * np.eye(n)
        assert np.allclose(cholesky(spd), np.linalg.cholesky(spd), atol=1e-12)
    with pytest.raises(NotPositiveDefinite):
        cholesky(W.corr_equi(3, -0.6))


def test_gbm_zero_vol_is_deterministic_growth():
    days = [3, 10, 252]
    z = np.random.default_rng(1).normal(size=(4, 3, 2))
    S = gbm_paths(z, days, 1 / 252, 0.05, [100.0, 50.0], [0.0, 0.0], np.eye(2))
    for s, d in enumerate(days):
        assert np.allclose(S[:, s, 0], 100 * math.exp(0.05 * d / 252), rtol=1e-14)
        assert np.allclose(S[:, s, 1], 50 * math.exp(0.05 * d / 252), rtol=1e-14)


def test_gbm_log_return_moments_and_correlation():
    p = problem(W.C2, rng="philox")
    S = p.paths(np.arange(20000))
    lr = np.log(S[:, 0, :] / 100.0)          # one year
    vol = np.array(W.C2.vol)
    assert np.allclose(lr.mean(0), 0.03 - 0.5 * vol**2, atol=4 * vol.max() / math.sqrt(20000))
    assert np.allclose(lr.std(0, ddof=1), vol, rtol=0.03)
    r = np.corrcoef(lr.T)
    assert np.allclose(r[np.triu_indices(3, 1)], 0.5, atol=0.03)


def test_estimate_matches_numpy():
    x = np.random.default_rng(2).normal(3, 2, size=1001)
    m, se = mc.estimate(x)
    assert m == pytest.approx(x.mean(), rel=1e-14)
    assert se == pytest.approx(x.std(ddof=1) / math.sqrt(x.size), rel=1e-12)


def test_c1_matches_black_scholes():
    p = problem(W.C1)
    pay = p.payoffs(np.arange(1 << 14))
    m, se = mc.estimate(pay)
    bs = cf.bs_call(100, 100, 0.03, 0.2, 1.0)
    assert bs == pytest.approx(9.413403383853016, rel=1e-13)
    assert abs(m - bs) < 3 * se


def test_forward_and_cash_legs():
    fwd = "(mult (model S (tvar T)) (payoff (tvar T) X Y))"
    p = problem(W.C1, il=fwd)
    pay = p.payoffs(np.arange(1 << 13))
    m, se = mc.estimate(pay)
    assert abs(m - 100.0) < 3 * se                         # martingale
    cash = problem(W.C1, il="(mult (model K 0) (payoff (tvar T) X Y))")
    pay = cash.payoffs(np.arange(64))
    assert np.all(pay == 100 * math.exp(-0.03 * 252 * (1 / 252)))
    assert pay[0] == pytest.approx(97.04455335485082, rel=1e-15)


def test_down_and_out_special_cases_are_exact():
    """B -> 0 never knocks out: the value is the call on the same simulated
    days (direct numpy formula); B >= S0 knocks out on day 0: exactly 0."""
    ids = np.arange(256)
    base = problem(W.C3, tenv={"T": 300})
    vanilla = problem(W.C3, tenv={"T": 300}, params=[100.0, 0.0])
    S = vanilla.paths(ids)[:, :, 0]
    assert vanilla.days == list(range(1, 301))
    ref = np.maximum(S[:, -1] - 100.0, 0.0) * math.exp(-0.03 * 300 / 252)
    assert np.allclose(vanilla.payoffs(ids), ref, rtol=1e-15, atol=0)
    dead = problem(W.C3, tenv={"T": 300}, params=[100.0, 100.0])
    assert np.all(dead.payoffs(ids) == 0.0)
    pb = base.payoffs(ids)
    knocked = S.min(1) <= 70.0
    assert np.array_equal(pb, np.where(knocked, 0.0, vanilla.payoffs(ids)))


@pytest.mark.slow
def test_down_and_out_near_discrete_closed_form():
    """Quarter-year daily barrier: MC within 3 SE of the BGK-shifted
    continuous formula (which is accurate to far below the SE here)."""
    T = 63
    p = problem(W.C3, tenv={"T": T}, params=[100.0, 90.0])
    pay = p.payoffs(np.arange(1 << 13))
    m, se = mc.estimate(pay)
    bgk = cf.down_and_out_call(100, 100, cf.bgk_barrier(90, 0.3, 1 / 252), 0.03, 0.3, T / 252)
    cont = cf.down_and_out_call(100, 100, 90, 0.03, 0.3, T / 252)
    assert abs(m - bgk) < 3 * se
    assert m > cont - 3 * se


def test_closed_form_identities():
    c = cf.bs_call(100, 95, 0.03, 0.25, 2.0)
    assert c - cf.bs_put(100, 95, 0.03, 0.25, 2.0) == pytest.approx(100 - 95 * math.exp(-0.06), rel=1e-13)
    assert cf.down_and_out_call(100, 100, 1e-6, 0.03, 0.3, 5) == pytest.approx(cf.bs_call(100, 100, 0.03, 0.3, 5), rel=1e-12)
    assert cf.down_and_out_call(100, 100, 70, 0.03, 0.3, 5) == pytest.approx(26.6745, abs=1e-4)
    assert cf.down_and_out_call(100, 100, cf.bgk_barrier(70, 0.3, 1 / 252), 0.03, 0.3, 5) == pytest.approx(27.0184, abs=1e-4)
    assert cf.down_and_out_call(60, 100, 70, 0.03, 0.3, 5) == 0.0


def test_autocall_special_cases():
    ids = np.arange(512)
    # zero vol: S(1) = 100 e^0.03 >= 100, so it redeems on date 1
    p = problem(W.C2, vol=[0.0, 0.0, 0.0])
    assert np.allclose(p.payoffs(ids), 105 * math.exp(-0.03), rtol=1e-15)
    no_call_no_ki = W.WORST_OF_AUTOCALL.replace("(real 100.0) (min", "(real 1e300) (min").replace("(real 60.0)", "(real -1.0)")
    p = problem(W.C2, il=no_call_no_ki)
    assert np.allclose(p.payoffs(ids), 100 * math.exp(-0.15), rtol=1e-15)
    # no autocall, knock-in always, identical assets: pays S(5) d(5); E = 100
    always_ki = W.WORST_OF_AUTOCALL.replace("(real 100.0) (min", "(real 1e300) (min").replace("(real 60.0)", "(real 1e300)")
    # (perfect correlation is a singular matrix; use one asset three times)
    one = always_ki.replace("S2", "S1").replace("S3", "S1")
    p = problem(W.C2, il=one, asset_labels=["S1"], spot=[100.0], vol=[0.2], corr=None, rng="philox")
    pay = p.payoffs(np.arange(1 << 13))
    m, se = mc.estimate(pay)
    assert abs(m - 100.0) < 3 * se


def test_brute_force_barrier_call_tiny():
    """N <= 8 paths, 3 dates: the IL value equals a direct numpy formula."""
    il = ("(loopif (leq (model S 1) (model B 0)) (real 0.0) "
          "(if (lt (model K 0) (model S 1)) (mult (sub (model S 1) (model K 0)) (payoff 1 X Y)) (real 0.0)) 2)")
    for seed in range(5):
        p = problem(W.C3, il=il, tenv={}, params=[100.0, 85.0], seed=seed, vol=[0.5])
        S = p.paths(np.arange(8))[:, :, 0]             # days 1, 2, 3
        assert p.days == [1, 2, 3]
        d3 = math.exp(-0.03 * 3 / 252)
        ref = np.where(S.min(1) <= 85.0, 0.0, np.maximum(S[:, 2] - 100.0, 0.0) * d3)
        assert np.allclose(p.payoffs(np.arange(8)), ref, rtol=1e-15, atol=0)


def test_double_option_linearity():
    c1 = "(if (lt (model K 0) (model S1 (tvar T))) (mult (sub (model S1 (tvar T)) (model K 0)) (payoff (tvar T) X Y)) (real 0.0))"
    c2 = c1.replace("S1", "S2")
    kw = dict(asset_labels=["S1", "S2"], param_labels=["K"], params=[100.0], tenv={"T": 252}, spot=[100, 100],
              vol=[0.2, 0.3], corr=W.corr_equi(2, 0.5), rate=0.03, years_per_day=1 / 252)
    ids = np.arange(2048)
    both = mc.Problem(f"(add {c1} {c2})", **kw).payoffs(ids)
    a = mc.Problem(c1, **kw).payoffs(ids)
    b = mc.Problem(c2, **kw).payoffs(ids)
    assert np.array_equal(both, a + b)
    m, se = mc.estimate(both)
    ref = cf.bs_call(100, 100, 0.03, 0.2, 1.0) + cf.bs_call(100, 100, 0.03, 0.3, 1.0)
    assert abs(m - ref) < 3 * se


def test_sobol_and_philox_streams_agree_statistically():
    a = problem(W.C2)
    b = problem(W.C2, rng="philox")
    pa, pb = a.payoffs(np.arange(4096)), b.payoffs(np.arange(4096))
    ma, sa = mc.estimate(pa)
    mb, sb = mc.estimate(pb)
    assert abs(ma - mb) < 3 * math.hypot(sa, sb)


def test_double_call_is_sum_of_its_legs_and_black_scholes():
    """The double option is linear in its legs: on every path its payoff is
    the sum of the two calls' payoffs on the same correlated paths, and the
    price agrees with the sum of the two Black-Scholes prices within 4
    standard errors."""
    import math
    from oracle import closed_form as cf
    cfg = W.C2D
    n = 4096
    kw = dict(asset_labels=cfg.asset_labels, param_labels=cfg.param_labels, params=cfg.params,
              tenv=cfg.tenv_dict(), spot=cfg.spot, vol=cfg.vol, corr=cfg.corr, rate=cfg.rate,
              years_per_day=cfg.years_per_day, rng=cfg.rng, seed=cfg.seed, precision="f64")
    both = mc.Problem(cfg.il, **kw).payoffs(np.arange(n))
    leg = lambda a: (f"(if (lt (model K{a} 0) (model S{a} (tvar T))) "
                     f"(mult (sub (model S{a} (tvar T)) (model K{a} 0)) (payoff (tvar T) X Y)) (real 0.0))")
    legs = sum(mc.Problem(leg(a), **kw).payoffs(np.arange(n)) for a in (1, 2))
    assert np.allclose(both, legs, rtol=1e-15, atol=1e-12)
    p, se = mc.estimate(both)
    T = 252 / 252.0
    ref = cf.bs_call(100.0, 100.0, 0.03, 0.2, T) + cf.bs_call(100.0, 95.0, 0.03, 0.3, T)
    assert abs(p - ref) < 4 * se, (p, ref, se)
