"""Monte Carlo valuation of a payoff expression (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The method (Sec. 3 and Sec. 6.2): simulate scenarios of the external
environment, evaluate the compiled payoff expression on each, and aggregate.
Per path the steps are: random words -> uniforms -> normals -> correlated
normals -> GBM prices on the simulated days -> payoff value by the semantics
of Fig. 3 with t0 = 0 and the current time t = t_now -> one sum over paths.

Pricing at a current time with a price history (Sec. 4.1): the environment
is the union of historical data, for the days up to the current day, and
simulated data after it.  Given history[a][j], the price of asset a on day
t_now - n + 1 + j (j < n, so the history ends on the current day), a day up
to t_now reads the history (days before its first one read the first
value), and the simulation starts on day t_now from the history's last
prices; the discount function d stays the one of day 0 (Thm. 5).  Without a
history, days up to 0 read the spot and the simulation starts on day 0.

The estimate is the sample mean; the standard error is the sample standard
deviation (denominator N-1) over sqrt(N).  Sums use math.fsum.
"""
from __future__ import annotations

import math

import numpy as np

from . import grid
from .il import il_eval, parse, typeof
from .model import cholesky, discount, gbm_paths, inv_cdf
from .rng import philox_words, sobol_words, uniform_f32, uniform_f64


class Problem:
    """A payoff expression together with everything one pricing needs."""

    def __init__(self, il, *, asset_labels, param_labels=(), params=(), tenv=None,
                 spot, vol, corr=None, rate, years_per_day, rng="philox", seed=42,
                 instance=0, precision="f32", t_now=0, parties=("X", "Y"), history=None):
        self.ast = parse(il) if isinstance(il, str) else il
        self.asset_labels = list(asset_labels)
        self.param_labels = list(param_labels)
        self.params = dict(zip(self.param_labels, [float(x) for x in params]))
        typeof(self.ast, set(self.asset_labels) | set(self.param_labels))
        self.delta = dict(tenv or {})
        self.spot = np.asarray(spot, dtype=np.float64).reshape(-1)
        self.vol = np.asarray(vol, dtype=np.float64).reshape(-1)
        A = len(self.asset_labels)
        self.corr = np.eye(A) if corr is None else np.asarray(corr, dtype=np.float64).reshape(A, A)
        self.L = cholesky(self.corr)
        self.rate = float(rate)
        self.ypd = float(years_per_day)
        self.rng = rng
        self.seed = int(seed)
        self.instance = int(instance)
        self.precision = precision
        self.t_now = int(t_now)
        self.p1, self.p2 = parties
        self.history = None
        self.start = 0
        self.sim_spot = self.spot
        if history is not None:
            h = np.asarray(history, dtype=np.float64).reshape(A, -1)
            if self.t_now < 0 or h.shape[1] < 1 or not np.all(np.isfinite(h) & (h > 0)):
                raise ValueError("a history needs t_now >= 0 and finite positive prices")
            self.history = h
            self.hist_first = self.t_now - h.shape[1] + 1
            self.start = self.t_now
            self.sim_spot = h[:, -1].copy()
        self.days = grid.slots(self.ast, self.delta, self.asset_labels, after=self.start)
        self.slot_of = {d: s for s, d in enumerate(self.days)}
        self.d = discount(self.rate, self.ypd)

    @property
    def n_assets(self):
        return len(self.asset_labels)

    @property
    def n_words(self):
        return len(self.days) * self.n_assets

    # -- per-path pipeline ----------------------------------------------------
    def words(self, path_ids):
        if self.rng == "philox":
            return philox_words(path_ids, self.n_words, self.instance, self.seed)
        if self.rng == "sobol":
            return sobol_words(path_ids, self.n_words)
        raise ValueError(self.rng)

    def uniforms(self, words):
        return uniform_f64(words) if self.precision == "f64" else uniform_f32(words)

    def normals(self, path_ids):
        w = self.words(path_ids)
        if w.size == 0:
            return np.zeros((len(path_ids), len(self.days), self.n_assets))
        z = inv_cdf(self.uniforms(w))
        return z.reshape(len(path_ids), len(self.days), self.n_assets)

    def paths(self, path_ids):
        """S[p][slot][asset] in binary64."""
        z = self.normals(path_ids)
        return gbm_paths(z, self.days, self.ypd, self.rate, self.sim_spot, self.vol, self.L, start=self.start)

    def env(self, S_path):
        """rho(label, day) for one path: a day up to the simulation's start
        is history (the spot, flat, without a given history), a later day
        the path; a parameter observable is its constant value."""
        idx = {lab: a for a, lab in enumerate(self.asset_labels)}
        h = self.history

        def rho(label, day):
            if label in self.params:
                return self.params[label]
            a = idx[label]
            if day <= self.start:
                if h is None:
                    return float(self.spot[a])
                j = min(max(day - self.hist_first, 0), h.shape[1] - 1)
                return float(h[a][j])
            return float(S_path[self.slot_of[day]][a])

        return rho

    def payoff_value(self, S_path):
        v = il_eval(self.ast, self.env(S_path), self.delta, 0, self.t_now, self.d, self.p1, self.p2)
        return float(v)

    def payoffs(self, path_ids):
        S = self.paths(path_ids)
        return np.array([self.payoff_value(S[i]) for i in range(len(path_ids))])

    def payoffs_on_paths(self, S):
        """Payoffs on given prices S[p][slot][asset] (e.g. paths another
        implementation stored), so payoff arithmetic is checked alone."""
        return np.array([self.payoff_value(S[i]) for i in range(S.shape[0])])


def estimate(values):
    """(mean, standard error) with fsum; SE uses the N-1 sample variance."""
    x = [float(v) for v in values]
    n = len(x)
    if n == 0:
        return float("nan"), float("nan")
    mean = math.fsum(x) / n
    if n < 2:
        return mean, float("nan")
    var = math.fsum((v - mean) ** 2 for v in x) / (n - 1)
    return mean, math.sqrt(var / n)


def price(il, n_paths, **kw):
    """Price ``il`` over paths 0..n_paths-1; returns (price, se, payoffs)."""
    prob = Problem(il, **kw)
    ids = np.arange(n_paths, dtype=np.int64)
    pay = prob.payoffs(ids)
    p, se = estimate(pay)
    return p, se, pay
