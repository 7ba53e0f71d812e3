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
