"""Pins of the oracle's bump-and-revalue risk (common random numbers)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import mc, risk


def _euro_kw(**over):
    kw = dict(asset_labels=["S"], param_labels=["K"], params=[100.0], tenv={"T": 252}, corr=None,
              rate=0.03, years_per_day=1.0 / 252.0, rng="philox", seed=42, precision="f64")
    kw.update(over)
    return kw


def test_central_differences_exact_on_quadratic():
    """Central differences are exact for V(S, sigma) quadratic in each
    argument; this pins the scenario order and the difference formulas."""
    spot, vol, rel, k = [90.0, 110.0], [0.2, 0.3], 0.01, 0.02

    def V(s, v):   # 3 s1^2 + 2 s1 s2 - s2^2 + 5 v1^2 + v2 s1
        return 3 * s[0] ** 2 + 2 * s[0] * s[1] - s[1] ** 2 + 5 * v[0] ** 2 + v[1] * s[0]

    prices = [V(s, v) for s, v in risk.scenarios(spot, vol, rel, k)]
    g = risk.greeks_from_prices(prices, spot, rel, k)
    s1, s2, v1, v2 = spot[0], spot[1], vol[0], vol[1]
    assert g["delta"] == pytest.approx([6 * s1 + 2 * s2 + v2, 2 * s1 - 2 * s2], rel=1e-9)
    assert g["gamma"] == pytest.approx([6.0, -2.0], rel=1e-6)
    assert g["vega"] == pytest.approx([10 * v1, s1], rel=1e-9)
    assert len(prices) == 1 + 4 * 2


def test_forward_gamma_is_zero_pathwise():
    """Every path's forward value is linear in the spot (S_T = S_0 e^x), so
    the central second difference vanishes up to rounding."""
    g = risk.risk(W.FORWARD, 512, spot=[100.0], vol=[0.25], rel=0.01, k=0.01, **_euro_kw())
    P = g["payoffs"]
    per_path = (P[1] - 2 * P[0] + P[2]) / 1.0
    assert np.max(np.abs(per_path)) < 1e-9
    # and the forward's delta on each path is d(T) S_T / S_0
    h = 1.0
    d = math.exp(-0.03)
    per_delta = (P[1] - P[2]) / (2 * h)
    S_T = (P[0] / d + 100.0)
    assert np.allclose(per_delta, d * S_T / 100.0, rtol=1e-9)


def test_european_greeks_match_black_scholes():
    """Bump-and-revalue Greeks of a European call agree with the analytic
    Black-Scholes delta, gamma and vega within 4 standard errors of the
    pathwise differences (the same paths in every scenario)."""
    n, S, K, r, sig, T = 1 << 14, 100.0, 100.0, 0.03, 0.2, 1.0
    rel, k = 0.01, 0.01
    g = risk.risk(W.EUROPEAN_CALL, n, spot=[S], vol=[sig], rel=rel, k=k, **_euro_kw())
    P = g["payoffs"]
    h = rel * S
    d_path = (P[1] - P[2]) / (2 * h)
    g_path = (P[1] - 2 * P[0] + P[2]) / (h * h)
    v_path = (P[3] - P[4]) / (2 * k)
    for est, path, exact in ((g["delta"][0], d_path, cf.bs_call_delta(S, K, r, sig, T)),
                             (g["gamma"][0], g_path, cf.bs_call_gamma(S, K, r, sig, T)),
                             (g["vega"][0], v_path, cf.bs_call_vega(S, K, r, sig, T))):
        se = path.std(ddof=1) / math.sqrt(n)
        assert est == pytest.approx(path.mean(), rel=1e-12, abs=1e-12)
        assert abs(est - exact) < 4 * se, (est, exact, se)


def test_scenarios_share_streams():
    """All scenarios draw the same normals (common random numbers)."""
    ids = np.arange(64)
    base = mc.Problem(W.EUROPEAN_CALL, spot=[100.0], vol=[0.2], **_euro_kw())
    for s, v in risk.scenarios([100.0], [0.2], 0.01, 0.01):
        p = mc.Problem(W.EUROPEAN_CALL, spot=s, vol=v, **_euro_kw())
        assert np.array_equal(p.normals(ids), base.normals(ids))
