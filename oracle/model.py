"""Normals, correlation and GBM paths (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper does not describe the engine's path construction; this build
fixes (each reading is listed in the design notes):

* normals: z = Phi^-1(u), the inverse standard normal CDF.  The oracle uses
  the standard library's ``NormalDist.inv_cdf`` (Wichura's AS241, PPND16,
  in binary64).
* correlation: w = L z with L the lower Cholesky factor of the asset
  correlation matrix (textbook Cholesky-Banachiewicz, binary64).
* model: risk-neutral geometric Brownian motion with constant rate r and
  volatilities sigma_a, no dividends.  Between consecutive simulated days
  the log-price moves by (r - sigma_a^2/2) dt + sigma_a sqrt(dt) w_a, with
  dt = (day_s - day_{s-1}) * years_per_day and day_{-1} = the day the
  simulation starts from (0, or the current day when a price history is
  given, Sec. 4.1); the price is S0_a exp(x_a) with S0 the price on that
  day.  This is exact in distribution at the grid dates.
* discount: d(day) = exp(-r * day * years_per_day).
"""
from __future__ import annotations

import math
from statistics import NormalDist

import numpy as np

_ND = NormalDist()


def inv_cdf(u):
    """Phi^-1 element-wise (AS241 via the standard library)."""
    f = _ND.inv_cdf
    u = np.asarray(u, dtype=np.float64)
    return np.vectorize(f, otypes=[np.float64])(u) if u.ndim else np.float64(f(float(u)))


class NotPositiveDefinite(ValueError):
    pass


def cholesky(a):
    """Lower-triangular L with L L^T = a (Cholesky-Banachiewicz, binary64)."""
    a = [[float(x) for x in row] for row in a]
    n = len(a)
    L = [[0.0] * n for _ in range(n)]
    for i in range(n):
        for j in range(i + 1):
            s = a[i][j]
            for k in range(j):
                s -= L[i][k] * L[j][k]
            if i == j:
                if not s > 0.0:
                    raise NotPositiveDefinite(f"leading minor {i + 1} is not positive")
                L[i][i] = math.sqrt(s)
            else:
                L[i][j] = s / L[j][j]
    return np.array(L)


def step_coefficients(days, years_per_day, rate, vol, start=0):
    """Per-slot drift and diffusion: m[s][a] = (r - sigma_a^2/2) dt_s,
    v[s][a] = sigma_a sqrt(dt_s), dt_s = (day_s - day_{s-1}) * years_per_day,
    day_{-1} = start."""
    vol = np.asarray(vol, dtype=np.float64)
    m = np.zeros((len(days), vol.size))
    v = np.zeros((len(days), vol.size))
    prev = start
    for s, day in enumerate(days):
        dt = (day - prev) * years_per_day
        m[s] = (rate - 0.5 * vol * vol) * dt
        v[s] = vol * math.sqrt(dt)
        prev = day
    return m, v


def gbm_paths(z, days, years_per_day, rate, spot, vol, L, start=0):
    """Prices S[p][s][a] from normals z[p][s][a] (binary64); spot is the
    price on day `start`, where the simulation begins."""
    z = np.asarray(z, dtype=np.float64)
    spot = np.asarray(spot, dtype=np.float64)
    m, v = step_coefficients(days, years_per_day, rate, vol, start)
    n_paths, n_slots, n_assets = z.shape
    S = np.zeros_like(z)
    x = np.zeros((n_paths, n_assets))
    for s in range(n_slots):
        w = z[:, s, :] @ np.asarray(L).T          # w_a = sum_k L[a][k] z_k
        x = x + m[s] + v[s] * w
        S[:, s, :] = spot * np.exp(x)
    return S


def discount(rate, years_per_day):
    """d(day) = exp(-r * day * years_per_day)."""
    return lambda day: math.exp(-rate * day * years_per_day)
