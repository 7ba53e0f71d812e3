"""Closed-form prices used to pin the Monte Carlo oracle.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

These are textbook results, not from the paper:
* Black-Scholes-Merton European call and put (no dividends).
* Down-and-out call with continuous monitoring and barrier B <= K, no rebate
  (Merton 1973; Reiner & Rubinstein 1991; the form in Hull's "Options,
  Futures and Other Derivatives"): price = call - down-and-in call.
* Broadie, Glasserman & Kou (1997): a barrier monitored at spacing dt is
  priced approximately by the continuous formula with the barrier moved away
  from the spot, B * exp(-beta sigma sqrt(dt)), beta = -zeta(1/2)/sqrt(2 pi).
"""
from __future__ import annotations

import math
from statistics import NormalDist

_N = NormalDist().cdf
BGK_BETA = 0.5825971579390106   # -zeta(1/2) / sqrt(2*pi)


def bs_call(S, K, r, sigma, T):
    sq = sigma * math.sqrt(T)
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / sq
    d2 = d1 - sq
    return S * _N(d1) - K * math.exp(-r * T) * _N(d2)


def bs_put(S, K, r, sigma, T):
    return bs_call(S, K, r, sigma, T) - S + K * math.exp(-r * T)


def down_and_in_call(S, K, B, r, sigma, T):
    """Continuous down-and-in call, B <= K, S > B, no dividends."""
    lam = (r + 0.5 * sigma * sigma) / (sigma * sigma)
    sq = sigma * math.sqrt(T)
    y = math.log(B * B / (S * K)) / sq + lam * sq
    return (S * (B / S) ** (2 * lam) * _N(y)
            - K * math.exp(-r * T) * (B / S) ** (2 * lam - 2) * _N(y - sq))


def down_and_out_call(S, K, B, r, sigma, T):
    """Continuous down-and-out call, B <= K; 0 if the spot is at/below B."""
    if S <= B:
        return 0.0
    return bs_call(S, K, r, sigma, T) - down_and_in_call(S, K, B, r, sigma, T)


def bgk_barrier(B, sigma, dt):
    """Barrier shift for discrete monitoring (down barrier moves down)."""
    return B * math.exp(-BGK_BETA * sigma * math.sqrt(dt))


def _d1(S, K, r, sigma, T):
    return (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / (sigma * math.sqrt(T))


def bs_call_delta(S, K, r, sigma, T):
    """dC/dS = N(d1)."""
    return _N(_d1(S, K, r, sigma, T))


def bs_call_gamma(S, K, r, sigma, T):
    """d2C/dS2 = phi(d1) / (S sigma sqrt(T))."""
    return NormalDist().pdf(_d1(S, K, r, sigma, T)) / (S * sigma * math.sqrt(T))


def bs_call_vega(S, K, r, sigma, T):
    """dC/dsigma = S phi(d1) sqrt(T)."""
    return S * NormalDist().pdf(_d1(S, K, r, sigma, T)) * math.sqrt(T)
