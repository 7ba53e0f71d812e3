"""Shared helpers of the GPU parity tests: a device context, the oracle
problem for a workload, and the tie-band used when FP32 and FP64 paths may
take different decisions (a comparison within a relative margin)."""
import numpy as np

import workloads as W
from oracle import mc

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        import paper_2108_03076_amd as P
        _CTX = P.Context(0)
    return _CTX


def oracle_problem(cfg, **over):
    kw = dict(asset_labels=cfg.asset_labels, param_labels=cfg.param_labels, params=cfg.params,
              tenv=cfg.tenv_dict(), spot=cfg.spot, vol=cfg.vol, corr=cfg.corr, rate=cfg.rate,
              years_per_day=cfg.years_per_day, rng=cfg.rng, seed=cfg.seed, precision=cfg.precision,
              parties=cfg.parties)
    il = over.pop("il", cfg.il)
    kw.update(over)
    return mc.Problem(il, **kw)


def gpu_payoff(cfg, il=None):
    import paper_2108_03076_amd as P
    return P.Payoff(ctx(), il or cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)


def model_kw(cfg, **over):
    kw = dict(spot=cfg.spot, vol=cfg.vol, corr=cfg.corr, rate=cfg.rate, years_per_day=cfg.years_per_day)
    kw.update(over)
    return kw


def opts_kw(cfg, n_paths, **over):
    kw = dict(n_paths=n_paths, rng=cfg.rng, seed=cfg.seed, precision=cfg.precision, parties=cfg.parties)
    kw.update(over)
    return kw


def tie_band(prob, S, eps):
    """True for paths whose oracle payoff jumps when every price moves by a
    relative +-eps (a decision within eps of its threshold)."""
    base = prob.payoffs_on_paths(S)
    up = prob.payoffs_on_paths(S * (1 + eps))
    dn = prob.payoffs_on_paths(S * (1 - eps))
    scale = np.maximum(np.abs(base), 1.0)
    smooth = 10 * eps * (np.abs(base) + np.max(np.abs(S), axis=(1, 2)))
    return (np.abs(up - base) > smooth) | (np.abs(dn - base) > smooth) | (scale < 0)


def sample_ids(n, k, seed=0):
    g = np.random.default_rng(seed)
    ids = np.unique(np.concatenate([[0, 1, n - 1], g.integers(0, n, size=k)]))
    return ids.astype(np.int64)


_GOLDEN = None


def golden():
    """Stored oracle values (tests/golden/oracle_values.json, written by
    tests/golden/make_oracle_values.py from the oracle alone)."""
    global _GOLDEN
    if _GOLDEN is None:
        import json
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")
        with open(path) as f:
            _GOLDEN = json.load(f)
    return _GOLDEN


def band_cap(case, n, tail=1e-6):
    """(expected, cap) tie-band counts for n paths of a stored case.  The
    rate is the band count k of M independent oracle paths, taken at its
    upper bound (k + 3 sqrt(k) + 3) / M; the cap is the count a Poisson
    variable of that mean exceeds with probability below `tail`."""
    from scipy.stats import poisson
    r = golden()["band_rates"][case]
    k, m = r["band"], r["sample"]
    lam = n * (k + 3.0 * np.sqrt(k) + 3.0) / m
    return n * k / m, int(poisson.isf(tail, lam))


def check_band(case, band, n=None):
    """Prints the tie-band count of a per-path comparison and asserts that it
    is within the cap derived from the case's stored band rate (a band far
    above its expected size would make the comparison vacuous)."""
    n = band.size if n is None else n
    count = int(np.sum(band))
    exp, cap = band_cap(case, n)
    print(f"[tie-band] {case}: {count} of {n} paths (expected {exp:.2f}, cap {cap})", flush=True)
    assert count <= cap, (case, count, exp, cap)
    return count
