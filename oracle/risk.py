"""Bump-and-revalue risk on common random numbers (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper motivates pricing one compiled contract many times over: risk
runs are thousands of pricings of the same instrument (end of Sec. 6.2).  The Greeks
of one instrument are central differences of Monte Carlo prices under bumped
models, every scenario driven by the same random words (the same instance
counter and seed, hence the same normals):

    delta_a = (V(S_a + h_a) - V(S_a - h_a)) / (2 h_a),   h_a = rel * S_a
    gamma_a = (V(S_a + h_a) - 2 V + V(S_a - h_a)) / h_a^2
    vega_a  = (V(sigma_a + k) - V(sigma_a - k)) / (2 k)

Scenario order (shared with the library's batch layout): the base model,
then for each asset a the pair (S_a + h_a, S_a - h_a), then for each asset
the pair (sigma_a + k, sigma_a - k): 1 + 4A scenarios.
"""
from __future__ import annotations

import numpy as np

from . import mc


def scenarios(spot, vol, rel, k):
    """The 1 + 4A (spot, vol) pairs of one instrument, in scenario order."""
    spot = [float(x) for x in spot]
    vol = [float(x) for x in vol]
    out = [(list(spot), list(vol))]
    for a in range(len(spot)):
        h = rel * spot[a]
        for sg in (1.0, -1.0):
            s = list(spot)
            s[a] = spot[a] + sg * h
            out.append((s, list(vol)))
    for a in range(len(vol)):
        for sg in (1.0, -1.0):
            v = list(vol)
            v[a] = vol[a] + sg * k
            out.append((list(spot), v))
    return out


def greeks_from_prices(prices, spot, rel, k):
    """Central differences from the scenario prices (in scenario order)."""
    A = len(spot)
    V = prices[0]
    delta, gamma, vega = [], [], []
    for a in range(A):
        h = rel * float(spot[a])
        up, dn = prices[1 + 2 * a], prices[2 + 2 * a]
        delta.append((up - dn) / (2.0 * h))
        gamma.append((up - 2.0 * V + dn) / (h * h))
    for a in range(A):
        up, dn = prices[1 + 2 * A + 2 * a], prices[2 + 2 * A + 2 * a]
        vega.append((up - dn) / (2.0 * k))
    return {"price": V, "delta": delta, "gamma": gamma, "vega": vega}


def risk(il, n_paths, *, spot, vol, rel, k, **problem_kw):
    """Greeks of one instrument; also the per-path scenario payoffs
    [scenario][path] so that standard errors of the differences can be
    formed (the same paths in every scenario)."""
    ids = np.arange(n_paths, dtype=np.int64)
    pays = []
    for s, v in scenarios(spot, vol, rel, k):
        prob = mc.Problem(il, spot=s, vol=v, **problem_kw)
        pays.append(prob.payoffs(ids))
    prices = [mc.estimate(p)[0] for p in pays]
    g = greeks_from_prices(prices, spot, rel, k)
    g["scenario_prices"] = prices
    g["payoffs"] = np.array(pays)
    return g
