"""Writes tests/golden/oracle_values.json: values the GPU tests compare with,
computed by the FP64 oracle alone (nothing here calls the GPU library).

* Tie-band rates.  For each FP32 case whose per-path comparison excludes
  the tie-band (paths whose oracle payoff jumps when every price moves by a
  relative +-3e-5), the band count on an independent sample of paths.  The
  tests turn it into an expected count and a cap for their own path counts.
* The batched workload's sample instances (16 of the 1024 down-and-out
  calls spanning 252..1260 days) at 2^12 paths: price and standard error;
  the tie-band count and the largest payoff jump over the band (what FP32
  decisions near a barrier can move); and, as the pin for a vanishing
  barrier, the vanilla call max(S_T - K, 0) d(T) written directly on the
  same paths.
* Full-size instances (2^16 paths) of the same batch: price and standard
  error.
* The worst-of autocall at its full 2^20 Sobol paths: price and standard
  error.

Usage: python tests/golden/make_oracle_values.py [--procs 8]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
TESTS = os.path.dirname(HERE)
ROOT = os.path.dirname(TESTS)
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)

import numpy as np  # noqa: E402

EPS = 3e-5
# Per-case band samples: first path index and count (independent of the
# tests' own paths 0 .. n-1; Sobol cases stay low so that the oracle's
# generator need not produce millions of points first).
BAND_SAMPLE = {"c3_full": 4000}
BAND_DEFAULT = 20000
BAND_FIRST = 1 << 16
CHUNK = 2000


def _problem(cfg, **over):
    from gpu_common import oracle_problem
    return oracle_problem(cfg, **over)


def _band_chunk(args):
    name, lo, hi = args
    import warnings
    warnings.filterwarnings("ignore", message="The balance properties")
    from cases import BAND_CASES
    from gpu_common import tie_band
    cfg = BAND_CASES[name]
    prob = _problem(cfg)
    ids = np.arange(lo, hi)
    S = prob.paths(ids)
    return name, int(tie_band(prob, S, EPS).sum()), hi - lo


def _c4_chunk(args):
    idx, T, K, B, lo, hi, with_band = args
    import workloads as W
    cfg = W.C4
    prob = _problem(cfg, tenv={"T": int(T)}, params=[float(K), float(B)], instance=int(idx))
    ids = np.arange(lo, hi)
    S = prob.paths(ids)
    pay = prob.payoffs_on_paths(S)
    out = {"sum": math.fsum(pay), "sum_sq": math.fsum(pay * pay), "n": hi - lo}
    # vanilla call on the same paths, written directly (no IL): the last
    # simulated day is T
    ST = S[:, -1, 0]
    van = np.maximum(ST - K, 0.0) * math.exp(-cfg.rate * T * cfg.years_per_day)
    out["vanilla_sum"] = math.fsum(van)
    out["vanilla_sum_sq"] = math.fsum(van * van)
    if with_band:
        up = prob.payoffs_on_paths(S * (1 + EPS))
        dn = prob.payoffs_on_paths(S * (1 - EPS))
        jump = np.maximum(np.abs(up - pay), np.abs(dn - pay))
        smooth = 10 * EPS * (np.abs(pay) + np.max(np.abs(S), axis=(1, 2)))
        band = jump > smooth
        out["band"] = int(band.sum())
        out["band_jump_max"] = float(jump[band].max()) if band.any() else 0.0
        out["band_jump_sum"] = float(jump[band].sum())
    return idx, out


def _se(s, ss, n):
    var = max(0.0, (ss - s * s / n) / (n - 1))
    return math.sqrt(var / n)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=os.path.join(HERE, "oracle_values.json"))
    args = ap.parse_args()
    from cases import BAND_CASES, C4_FULL_PICK, C4_SAMPLE_PATHS, c4_sample

    t0 = time.time()
    tasks = []
    for name in BAND_CASES:
        m = BAND_SAMPLE.get(name, BAND_DEFAULT)
        first = BAND_FIRST
        if BAND_CASES[name].rng == "sobol":
            first = 4096
        for lo in range(first, first + m, CHUNK):
            tasks.append(("band", (name, lo, min(first + m, lo + CHUNK))))
    ids, T, K, B = c4_sample()
    n4 = C4_SAMPLE_PATHS
    for i in range(ids.size):
        for lo in range(0, n4, 1024):
            tasks.append(("c4", (int(ids[i]), int(T[i]), float(K[i]), float(B[i]), lo, lo + 1024, True)))
    # full size: the shortest, the longest and evenly spaced ranks between
    fids, fT, fK, fB = c4_sample(C4_FULL_PICK)
    nf = 1 << 16
    for i in range(fids.size):
        for lo in range(0, nf, 4096):
            tasks.append(("c4full", (int(fids[i]), int(fT[i]), float(fK[i]), float(fB[i]), lo, lo + 4096, False)))
    # the worst-of autocall over all 2^20 Sobol points
    n2 = 1 << 20
    for lo in range(0, n2, 1 << 16):
        tasks.append(("c2full", (lo, lo + (1 << 16))))
    # longest tasks first
    weight = {"band": 1, "c2full": 1, "c4": 2, "c4full": 3}
    tasks.sort(key=lambda t: -weight[t[0]])

    with Pool(args.procs) as pool:
        results = pool.map(_dispatch, tasks, chunksize=1)

    band = {}
    c2s = [0.0, 0.0, 0]
    c4 = {}
    c4f = {}
    for kind, res in results:
        if kind == "c2full":
            c2s[0] += res[0]; c2s[1] += res[1]; c2s[2] += res[2]
        elif kind == "band":
            name, k, m = res
            b = band.setdefault(name, {"band": 0, "sample": 0})
            b["band"] += k
            b["sample"] += m
        else:
            idx, out = res
            acc = (c4 if kind == "c4" else c4f).setdefault(idx, {})
            for key, v in out.items():
                if key == "band_jump_max":
                    acc[key] = max(acc.get(key, 0.0), v)
                else:
                    acc[key] = acc.get(key, 0) + v
    rec = {
        "generated_by": "tests/golden/make_oracle_values.py (FP64 oracle only)",
        "band_eps": EPS,
        "band_rates": {k: {**v, "first_path": 4096 if BAND_CASES[k].rng == "sobol" else BAND_FIRST}
                       for k, v in sorted(band.items())},
        "c4_sample": {"paths": n4, "instances": []},
        "c4_full": {"paths": nf, "instances": []},
        "c2_full_price": {"paths": c2s[2], "price": c2s[0] / c2s[2], "se": _se(c2s[0], c2s[1], c2s[2])},
    }
    for key, src, sel in (("c4_sample", c4, (ids, T, K, B)), ("c4_full", c4f, (fids, fT, fK, fB))):
        for i in range(sel[0].size):
            idx = int(sel[0][i])
            a = src[idx]
            n = a["n"]
            e = {"id": idx, "T": int(sel[1][i]), "K": float(sel[2][i]), "B": float(sel[3][i]),
                 "price": a["sum"] / n, "se": _se(a["sum"], a["sum_sq"], n), "sum": a["sum"],
                 "sum_sq": a["sum_sq"], "vanilla_price": a["vanilla_sum"] / n,
                 "vanilla_se": _se(a["vanilla_sum"], a["vanilla_sum_sq"], n)}
            for extra in ("band", "band_jump_max", "band_jump_sum"):
                if extra in a:
                    e[extra] = a[extra]
            rec[key]["instances"].append(e)
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {args.out} in {time.time() - t0:.0f} s")


def _c2_chunk(args):
    lo, hi = args
    import workloads as W
    prob = _problem(W.C2)
    pay = prob.payoffs(np.arange(lo, hi))
    return math.fsum(pay), math.fsum(pay * pay), hi - lo


def _dispatch(t):
    import warnings
    warnings.filterwarnings("ignore", message="The balance properties")
    if t[0] == "band":
        return t[0], _band_chunk(t[1])
    if t[0] == "c2full":
        return t[0], _c2_chunk(t[1])
    return t[0], _c4_chunk(t[1])


if __name__ == "__main__":
    main()
