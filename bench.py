#!/usr/bin/env python3
"""Throughput benchmark: path-dates per second priced on one MI355X.

Headline workload (the `value` of the JSON line): the worst-of autocall on 3
correlated assets, 5 annual dates, 2^20 unscrambled Sobol paths, FP32 paths
with an FP64 path sum.  One step = one complete pmc_price call (Cholesky
factor on the device, fused generate-and-evaluate kernel, deterministic
reduction, 16-byte result back to the host), with every input resident on
the device or in the call's small host structs.

Extra workloads (same JSON line, key "workloads"): the FP64 European call,
the 1260-day down-and-out call (fused, and two-phase with stored paths), and
the batched 1024-instance graph replay.  The CPU baseline is the FP64
oracle, single-threaded, on a bounded sample of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (dense) and the VALU issue rate the ALU roofline uses:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per second.
METRIC = "path-dates/sec priced (plain MC vs batched/surrogate at \u22640.5% err), % roofline"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 39.3 T lane-ops/s

# Algorithmic lane-operations per asset-date of path generation (FP32), by
# component; the design notes derive each figure.
OPS_UNIFORM = 2          # shift, int->float fused with scale and offset
OPS_NORMAL = 11          # AS241 PPND7 central branch: 2 + 4 + 3 + rcp + mul
OPS_STEP = 2             # drift and diffusion FMAs
OPS_EXP = 3              # scale by log2(e), exp2, times spot
OPS_SOBOL = 1            # one XOR per point with Gray-code stepping
OPS_PHILOX = 15          # 10 rounds x (2 mul-hi, 2 mul-lo, 2 xor3) / 4 words


# HBM traffic of the headline kernel per launch, from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE: KiB per dispatch) scaled by what the same
# counters read for a 256 MiB device-to-device copy in the same run (FETCH
# reads 0.5 KiB per KiB copied, WRITE 1.0).  Valid only for the engine sources
# it was measured on (hash below); otherwise reported as null.
TRAFFIC = {"engine_sha256": "ede50bd7b91d2ec53d224d7c94d5f44f56ed96dd5820e60f04dea5240c8170fc",
           "fetch_kib": 1225.0, "write_kib": 64.0, "fetch_scale": 2.0, "write_scale": 1.0}
ENGINE_SOURCES = ("paper_2108_03076_amd/csrc/mc_engine.h", "paper_2108_03076_amd/csrc/pmc_device.h",
                  "paper_2108_03076_amd/csrc/codegen.cpp")


def engine_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ENGINE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    t = TRAFFIC
    if t["engine_sha256"] is None or t["engine_sha256"] != engine_sha256():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def ops_per_path_date(n_assets, rng, il_ops_per_date):
    word = OPS_SOBOL if rng == "sobol" else OPS_PHILOX
    corr = (n_assets + 1) / 2 if n_assets > 1 else 0
    per_asset = word + OPS_UNIFORM + OPS_NORMAL + corr + OPS_STEP + OPS_EXP
    return n_assets * per_asset + il_ops_per_date


def _sync():
    import torch
    torch.cuda.synchronize()


def time_steps(fn, steps, warmup):
    for _ in range(warmup):
        fn()
    _sync()
    t0 = time.perf_counter()
    outs = [fn() for _ in range(steps)]
    _sync()
    return (time.perf_counter() - t0) / steps, outs


def cpu_baseline(cfg, n_paths):
    from oracle import mc
    import numpy as np
    prob = mc.Problem(cfg.il, asset_labels=cfg.asset_labels, param_labels=cfg.param_labels,
                      params=cfg.params, tenv=cfg.tenv_dict(), spot=cfg.spot, vol=cfg.vol, corr=cfg.corr,
                      rate=cfg.rate, years_per_day=cfg.years_per_day, rng=cfg.rng, seed=cfg.seed,
                      precision=cfg.precision)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):      # one core: BLAS and OpenMP pools pinned to one thread
        t0 = time.perf_counter()
        pay = prob.payoffs(np.arange(n_paths))
        mc.estimate(pay)
        dt = time.perf_counter() - t0
    return n_paths * len(prob.days) / dt, dt


def _oracle_chunk(args):
    cfg_name, lo, hi = args
    import warnings
    warnings.filterwarnings("ignore", message="The balance properties")   # partial Sobol ranges
    import numpy as np
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import mc
    cfg = W.CONFIGS[cfg_name]
    prob = mc.Problem(cfg.il, asset_labels=cfg.asset_labels, param_labels=cfg.param_labels,
                      params=cfg.params, tenv=cfg.tenv_dict(), spot=cfg.spot, vol=cfg.vol, corr=cfg.corr,
                      rate=cfg.rate, years_per_day=cfg.years_per_day, rng=cfg.rng, seed=cfg.seed,
                      precision=cfg.precision)
    with threadpool_limits(limits=1):
        pay = prob.payoffs(np.arange(lo, hi))
    return float(pay.sum()), len(prob.days)


def cpu_baseline_all_cores(cfg, n_paths):
    """The oracle over all host cores: contiguous path ranges in separate
    processes (exact, since the streams are counter based and indexable)."""
    import multiprocessing as mp
    n = min(os.cpu_count() or 1, 16)
    bounds = [(cfg_key(cfg), i * n_paths // n, (i + 1) * n_paths // n) for i in range(n)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(n) as pool:
        res = pool.map(_oracle_chunk, bounds)
    dt = time.perf_counter() - t0
    return n_paths * res[0][1] / dt, dt, n


def cfg_key(cfg):
    import workloads as W
    return next(k for k, v in W.CONFIGS.items() if v is cfg)


def surrogate_workload(ctx, args):
    """Labels from the batched Monte Carlo engine (2^16 Philox paths per
    point), training on the GPU, the Monte Carlo judge (2^22 paths, another
    seed) on held-out points, and inference against Monte Carlo timing."""
    import numpy as np
    import torch

    import paper_2108_03076_amd as P
    from paper_2108_03076_amd import surrogate as S
    import workloads as W

    c5 = W.C5
    pay = P.Payoff(ctx, c5.il, c5.asset_labels, c5.param_labels, c5.tvars)
    box = W.C5_BOX
    lo = [box["spot"][0]] * 3 + [box["vol"][0]] * 3 + [box["rho"][0], box["n_obs"][0]]
    hi = [box["spot"][1]] * 3 + [box["vol"][1]] * 3 + [box["rho"][1], box["n_obs"][1]]
    rec = {}
    n_train = args.surrogate_points
    xtr = W.c5_points(n_train, 42)
    t0 = time.perf_counter()
    ytr, setr, pd_tr, ms_tr = S.mc_prices(pay, xtr, c5.n_paths, rate=c5.rate, years_per_day=c5.years_per_day,
                                          seed=42)
    rec["label_gen_s"] = time.perf_counter() - t0
    rec["label_gen_gpu_ms"] = ms_tr
    rec["label_path_dates"] = int(pd_tr)
    rec["label_path_dates_per_s_gpu"] = pd_tr / (ms_tr * 1e-3)
    rec["label_rel_se_median"] = float(np.median(setr / ytr))
    n_test = c5.notes["test_points"]
    xte = W.c5_points(n_test, 43)
    t0 = time.perf_counter()
    yte, sete, pd_te, ms_te = S.mc_prices(pay, xte, c5.notes["judge_paths"], rate=c5.rate,
                                          years_per_day=c5.years_per_day, seed=43)
    rec["judge_s"] = time.perf_counter() - t0
    rec["judge_rel_se_median"] = float(np.median(sete / yte))
    sur = P.Surrogate(ctx, lo, hi, y_scale=100.0, width=256, seed=1)
    xt = torch.tensor(xtr, dtype=torch.float32, device="cuda")
    yt = torch.tensor(ytr, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    losses = S.train(sur, xt, yt, epochs=args.surrogate_epochs, batch=args.surrogate_batch,
                     lr_max=args.surrogate_lr, lr_min=1e-5)
    torch.cuda.synchronize()
    rec["train_s"] = time.perf_counter() - t0
    rec["train_epochs_batch_lr"] = [args.surrogate_epochs, args.surrogate_batch, args.surrogate_lr]
    rec["train_loss_first_last"] = [losses[0], losses[-1]]
    pred = torch.empty(n_test, dtype=torch.float32, device="cuda")
    sur.infer(torch.tensor(xte, dtype=torch.float32, device="cuda"), pred)
    rec["error_vs_judge"] = S.errors(pred.cpu().numpy(), yte)
    rec["error_plain_mc_2^16_vs_judge"] = S.errors(
        S.mc_prices(pay, xte, c5.n_paths, rate=c5.rate, years_per_day=c5.years_per_day, seed=44)[0], yte)
    nb = c5.notes["infer_batch"]
    xb = torch.tensor(W.c5_points(nb, 45), dtype=torch.float32, device="cuda")
    inf_ms, _ = S.timed_infer(sur, xb)
    rec["infer_batch"] = nb
    rec["infer_ms"] = inf_ms
    flop = 2.0 * (8 * 256 + 2 * 256 * 256 + 256) * nb
    rec["infer_roofline"] = {"bound": "mfma", "achieved": flop / (inf_ms * 1e-3) / 1e12, "peak": 2500.0,
                             "unit": "TFLOP/s (bf16 dense)", "frac": flop / (inf_ms * 1e-3) / 2.5e15}
    # Monte Carlo time for the same batch at 2^16 paths, from the label run's
    # device throughput; and at the paths giving the surrogate's RMS error
    mc_ms_2_16 = nb / n_train * ms_tr
    rec["mc_2^16_ms_same_batch"] = mc_ms_2_16
    rec["speedup_vs_mc_2^16"] = mc_ms_2_16 / inf_ms
    rel_se_2_16 = rec["label_rel_se_median"]
    err = max(rec["error_vs_judge"]["rms"], 1e-9)
    paths_eq = c5.n_paths * (rel_se_2_16 / err) ** 2
    rec["mc_paths_at_equal_error"] = paths_eq
    rec["speedup_vs_mc_equal_error"] = (mc_ms_2_16 * paths_eq / c5.n_paths) / inf_ms
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="headline workload only, no CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate workload")
    ap.add_argument("--only", default="",
                    help="comma-separated subset of the extra workloads to run (C1, C2i, C3, C4, risk, C5); "
                         "the headline always runs")
    ap.add_argument("--surrogate-points", type=int, default=1 << 20,
                    help="training points of the surrogate (each priced by Monte Carlo with 2^16 paths)")
    ap.add_argument("--surrogate-epochs", type=int, default=60)
    ap.add_argument("--surrogate-batch", type=int, default=4096)
    ap.add_argument("--surrogate-lr", type=float, default=2e-3, help="peak of the cosine learning-rate schedule")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also copy 256 MiB device-to-device three times (a known-size kernel for "
                         "scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in the design notes, not built)"}))
        sys.exit(2)

    # The oracle's CPU timings run first, before this process touches the
    # GPU (the all-cores run starts worker processes).
    import workloads as W
    cpu = None
    if not args.quick and not args.no_cpu_baseline:
        n_cpu = 1 << 20
        v, dt = cpu_baseline(W.C2, n_cpu)
        va, dta, ncores = cpu_baseline_all_cores(W.C2, n_cpu)
        cpu = (n_cpu, v, dt, va, dta, ncores)

    import numpy as np
    import torch

    import paper_2108_03076_amd as P

    ctx = P.Context(0)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def setup(cfg):
        pay = P.Payoff(ctx, cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)
        kw = dict(spot=cfg.spot, vol=cfg.vol, corr=cfg.corr, rate=cfg.rate, years_per_day=cfg.years_per_day,
                  n_paths=cfg.n_paths, rng=cfg.rng, seed=cfg.seed, precision=cfg.precision)
        return pay, kw

    # ---------------- headline: C2 worst-of autocall, fused ----------------
    c2 = W.C2
    pay2, kw2 = setup(c2)
    pricer = P.Pricer(pay2, c2.tenv, c2.params, **kw2)
    def step():                      # one pricing; keep only the two device times per step
        r = pricer()
        return (r.eval_ms, r.ms)
    sec, times = time_steps(step, args.steps, args.warmup)
    last = pricer.r.as_dict()          # the last timed step's full result
    D = last["n_slots"]
    pd = c2.n_paths * D
    value = pd / sec
    kern_ms = float(np.mean([t[0] for t in times]))
    # IL operations per date of the autocall: loop condition (2 min + 1 leq)
    # plus the maturity branch's knock-in checks spread over the dates.
    il_ops = 3 + (5 * 3 + 4 + 2) / D
    ops = ops_per_path_date(3, "sobol", il_ops) * pd
    achieved = ops / (kern_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "path-dates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Sobol stream, model parameters of the workload)",
        "config": {"workload": "worst-of autocall, 3 correlated assets (rho 0.5), 5 annual dates, "
                               "2^20 Sobol paths, FP32 paths, FP64 sum",
                   "paths": c2.n_paths, "dates": D, "assets": 3, "rng": "sobol", "mode": "fused"},
        "price": last["price"], "std_err": last["std_err"],
        "device_ms_per_step": float(np.mean([t[1] for t in times])),
        "engine": "compiled payoff (hipRTC)",
        # kernel_ms: the library's events from the start marker to the end of
        # the generated pricing kernel pmc_jit_mc (its launch gap included;
        # the one-block k_finish that follows is not)
        "roofline": {"bound": "alu", "kernel": "pmc_jit_mc<float,sobol,3 assets> (fused, compiled payoff)",
                     "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "T lane-op/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(),
                     "kernel_ms": kern_ms, "algorithmic_ops_per_launch": ops},
    }

    extra = {}
    only = set(x.strip() for x in args.only.split(",") if x.strip())
    want = lambda name: not args.quick and (not only or name in only)
    if want("C1"):
        # C1: FP64 European call (latency-bound at 2^16 paths)
        c1 = W.C1
        pay1, kw1 = setup(c1)
        s1, o1 = time_steps(lambda: P.price(pay1, c1.tenv, c1.params, **kw1), args.steps, args.warmup)
        extra["C1_fp64_european"] = {"ms_per_step": s1 * 1e3, "path_dates_per_s": c1.n_paths / s1,
                                     "kernel_ms": float(np.mean([o["eval_ms"] for o in o1])),
                                     "price": o1[-1]["price"], "std_err": o1[-1]["std_err"]}
    if want("C1"):
        # C1 swept over the path count (2^23 is the paper's vanilla size):
        # launch-latency bound at 2^16, FP64-arithmetic bound at the top
        from oracle.closed_form import bs_call
        ref = bs_call(100.0, 100.0, c1.rate, 0.2, 1.0)
        sweep = {}
        for lg in (16, 18, 20, 23, 26):
            kwn = dict(kw1, n_paths=1 << lg)
            sn, on = time_steps(lambda: P.price(pay1, c1.tenv, c1.params, **kwn), 5, 1)
            sweep[f"2^{lg}"] = {"ms_per_step": sn * 1e3, "path_dates_per_s": (1 << lg) / sn,
                                "kernel_ms": float(np.mean([o["eval_ms"] for o in on])),
                                "error_vs_black_scholes_in_se": (on[-1]["price"] - ref) / on[-1]["std_err"]}
        extra["C1_fp64_european_sweep"] = sweep
    if want("C2D"):
        # the double option: two calls on a correlated two-asset model
        c2d = W.C2D
        pay2d, kw2d = setup(c2d)
        sd, od = time_steps(lambda: P.price(pay2d, c2d.tenv, c2d.params, **kw2d), args.steps, args.warmup)
        extra["C2D_double_call"] = {"ms_per_step": sd * 1e3, "path_dates_per_s": c2d.n_paths / sd,
                                    "kernel_ms": float(np.mean([o["eval_ms"] for o in od])),
                                    "price": od[-1]["price"], "std_err": od[-1]["std_err"]}
    if want("C2i"):
        # the headline workload with the bytecode interpreter instead of the
        # compiled payoff
        si, oi = time_steps(lambda: P.price(pay2, c2.tenv, c2.params, engine="interpreter", **kw2),
                            max(3, args.steps // 4), 1)
        extra["C2_interpreter"] = {"ms_per_step": si * 1e3, "path_dates_per_s": pd / si,
                                   "kernel_ms": float(np.mean([o["eval_ms"] for o in oi]))}
    if want("C3"):
        # C3: 1260-day down-and-out call, fused and two-phase
        c3 = W.C3
        pay3, kw3 = setup(c3)
        for mode, engine in (("fused", "compiled"), ("two_phase", "compiled"), ("two_phase", "interpreter")):
            s3, o3 = time_steps(lambda: P.price(pay3, c3.tenv, c3.params, mode=mode, engine=engine, **kw3),
                                max(3, args.steps // 4), 1)
            pd3 = c3.n_paths * o3[-1]["n_slots"]
            rec = {"ms_per_step": s3 * 1e3, "path_dates_per_s": pd3 / s3,
                   "eval_ms": float(np.mean([o["eval_ms"] for o in o3])),
                   "gen_ms": float(np.mean([o["gen_ms"] for o in o3])),
                   "price": o3[-1]["price"], "std_err": o3[-1]["std_err"]}
            if mode == "two_phase":
                # the evaluator reads 4 B per path-date of stored prices
                gbs = 4.0 * pd3 / (rec["eval_ms"] * 1e-3) / 1e9
                rec["eval_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                                        "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
                gen_gbs = 4.0 * pd3 / (rec["gen_ms"] * 1e-3) / 1e9
                rec["gen_write_GBs"] = gen_gbs
            extra[f"C3_down_and_out_{mode}_{engine}"] = rec
    if want("C4") or want("risk"):
        # C4: 1024 templated instances, one persistent launch from a graph
        c4 = W.C4
        pay4, kw4 = setup(c4)
        T, K, B = W.c4_instances(1024, 42)
        tenv = T.reshape(-1, 1)
        params = np.stack([K, B], 1)
        bl, ppt = P.autotune_batch(pay4, tenv, params, **kw4)
    if want("C4"):
        s4, o4 = time_steps(lambda: P.price_batch(pay4, tenv, params, **kw4), max(3, args.steps // 4), 1)
        pd4 = int(sum(r["path_dates"] for r in o4[-1]))
        extra["C4_batched_1024"] = {"ms_per_step": s4 * 1e3, "path_dates_per_s": pd4 / s4,
                                    "graph_ms": float(np.mean([r[0]["ms"] for r in o4])),
                                    "path_dates": pd4, "tuned_block": bl, "tuned_paths_per_thread": ppt}
    if want("risk"):
        # Risk: delta, gamma and vega of the same 1024 instruments by central
        # differences on common random numbers, 1 + 4A = 5 scenarios each in
        # one persistent launch
        bumps = W.RISK_BUMPS
        sr, orr = time_steps(lambda: P.risk_batch(pay4, tenv, params, **bumps, **kw4), max(2, args.steps // 10), 1)
        n_scen = 1024 * 5
        pd_r = int(sum(r["path_dates"] for r in P.price_batch(pay4, tenv, params, **kw4))) * 5
        extra["C4_risk_1024x5"] = {"ms_per_step": sr * 1e3, "pricings_per_s": n_scen / sr,
                                   "greeks_per_s": 3 * 1024 / sr, "path_dates_per_s": pd_r / sr,
                                   "graph_ms": float(np.mean([r[0]["ms"] for r in orr])),
                                   "bumps": bumps, "instrument_0": orr[-1][0]}
    if want("C5") and not args.no_surrogate:
        extra["C5_surrogate"] = surrogate_workload(ctx, args)
    line["workloads"] = extra

    if cpu is not None:
        n_cpu, v, dt, va, dta, ncores = cpu
        line["cpu_oracle_all_cores"] = {"value": va, "unit": "path-dates/s", "cores": ncores,
                                        "seconds": dta, "paths": n_cpu}
        line["cpu_baseline"] = {"value": v, "unit": "path-dates/s", "cores": 1, "kind": "oracle",
                                "sample": f"first {n_cpu} of the 2^20 Sobol paths of the headline workload "
                                          f"({dt:.1f} s, FP64 numpy, one thread)",
                                "host": platform.processor() or platform.machine(),
                                "cpu_count": os.cpu_count()}
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
