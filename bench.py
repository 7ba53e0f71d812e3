#!/usr/bin/env python3
"""Throughput benchmark: path-dates per second priced on one MI355X.

Headline workload (the `value` of the JSON line): 1024 templated
down-and-out calls (daily monitoring over 252..1260 days, strike and
barrier per instance) of one loaded payoff expression, 2^16 Philox paths
each, priced as one persistent launch replayed from a HIP graph at the
autotuned tile.  One step = one complete pmc_price_batch call (host tables,
graph replay, per-instance FP64 reduction, 1024 results back on the host).
Inputs are resident: the model and the instances' parameters live in the
call's host arrays and are uploaded by the call itself.

Each price is reported with its error against the FP64 oracle on the same
random stream.  The CPU baseline is that oracle, single-threaded, on a
bounded sample of the headline workload (4 of its instances at 2^12 paths).

Extra workloads (key "workloads" of the same line): the worst-of autocall
(3 correlated assets, 2^20 Sobol paths), the FP64 European call and its
sweep to 2^26 paths (with and without the time guards of cutPayoff), the
double call, the 1260-day down-and-out (fused; two-phase with stored
paths), the risk batch and the learned surrogate.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "path-dates/sec priced (plain MC vs batched/surrogate at ≤0.5% err), % roofline"
# MI355X published peaks: HBM3E 8 TB/s; full-rate vector issue 256 CUs x 4
# SIMDs x 16 lanes x 2.4 GHz lane-operations per second (the rate of FP64
# FMA, and of FP32 without packed instructions).
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 39.3 T lane-ops/s

# Algorithmic lane-operations of path generation per asset-date (FP32), by
# component; the design notes derive each figure.
OPS_UNIFORM = 2          # shift, int->float fused with scale and offset
OPS_NORMAL = 11          # AS241 PPND7 central branch: 2 + 4 + 3 + rcp + mul
OPS_STEP = 2             # drift and diffusion FMAs
OPS_EXP = 3              # scale by log2(e), exp2, times spot
OPS_SOBOL = 1            # one XOR per point with Gray-code stepping
OPS_PHILOX = 15          # 10 rounds x (2 mul-hi, 2 mul-lo, 2 xor3) / 4 words
# Payoff operations per date of the down-and-out call: the barrier
# comparison, take = not done and hit, result select, done |= hit.
OPS_IL_DOWN_AND_OUT = 4

# HBM traffic of the headline kernel per launch, from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE: KiB per dispatch of the batched
# down-and-out kernel at the tuned tile, mean of the run's two dispatches)
# scaled by what the same counters read for the 256 MiB device-to-device
# copies of the same run (FETCH reads 0.5 KiB per KiB copied, WRITE 1.0;
# profiles/pmc_jit_mc_batched_down_and_out_counters.md).  Valid only for the
# engine sources it was measured on (hash below); otherwise reported as null.
TRAFFIC = {"engine_sha256": "2df20d5f431831c0387d04c1c070a19a125fcd6f54ab782bacffad2fcdf27fbb",
           "fetch_kib": 17515.8, "write_kib": 6223.8, "fetch_scale": 2.0, "write_scale": 1.0}
ENGINE_SOURCES = ("paper_2108_03076_amd/csrc/mc_engine.h", "paper_2108_03076_amd/csrc/pmc_device.h",
                  "paper_2108_03076_amd/csrc/codegen.cpp")
C4_CPU_SAMPLE = (4, 1 << 12)   # oracle baseline: instances, paths each


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


def err_vs(gpu_price, ref_price, ref_se):
    return {"gpu": gpu_price, "oracle": ref_price, "oracle_se": ref_se,
            "error_in_se": (gpu_price - ref_price) / ref_se if ref_se > 0 else None,
            "relative_error": (gpu_price - ref_price) / abs(ref_price) if ref_price else None}


# ----------------------------------------------------------------- oracle ---
def _oracle_problem(cfg, **over):
    from oracle import mc
    kw = dict(asset_labels=cfg.asset_labels, param_labels=cfg.param_labels, params=cfg.params,
              tenv=cfg.tenv_dict(), spot=cfg.spot, vol=cfg.vol, corr=cfg.corr, rate=cfg.rate,
              years_per_day=cfg.years_per_day, rng=cfg.rng, seed=cfg.seed, precision=cfg.precision)
    kw.update(over)
    return mc.Problem(cfg.il, **kw)


def _oracle_sums(args):
    """(sum, sum of squares, n, slots) of the oracle's payoffs over paths
    lo..hi-1 of one configuration (one process, one thread)."""
    cfg_name, over, lo, hi = args
    import warnings
    warnings.filterwarnings("ignore", message="The balance properties")   # partial Sobol ranges
    import numpy as np
    from threadpoolctl import threadpool_limits
    import workloads as W
    prob = _oracle_problem(W.CONFIGS[cfg_name], **over)
    with threadpool_limits(limits=1):
        pay = prob.payoffs(np.arange(lo, hi))
    return math.fsum(pay), math.fsum(pay * pay), hi - lo, len(prob.days)


def _estimate(s, ss, n):
    var = max(0.0, (ss - s * s / n) / (n - 1)) if n > 1 else 0.0
    return s / n, math.sqrt(var / n)


def c4_cpu_sample():
    """The oracle's sample of the headline workload: C4_CPU_SAMPLE[0]
    instances at evenly spaced ranks of their day count, first
    C4_CPU_SAMPLE[1] paths of each."""
    import numpy as np
    import workloads as W
    T, K, B = W.c4_instances(1024, 42)
    order = np.argsort(T, kind="stable")
    k, n = C4_CPU_SAMPLE
    ids = order[np.round(np.linspace(0, T.size - 1, k)).astype(int)]
    return [(int(i), int(T[i]), float(K[i]), float(B[i])) for i in ids], n


def _c4_over(i, T, K, B):
    return {"tenv": {"T": T}, "params": [K, B], "instance": i}


def cpu_baseline_c4():
    """The oracle on one core over the C4 sample, then the same sample split
    over the host's cores (exact: the streams are counter based)."""
    import multiprocessing as mp
    inst, n = c4_cpu_sample()
    t0 = time.perf_counter()
    one = [_oracle_sums(("C4", _c4_over(*e), 0, n)) for e in inst]
    dt1 = time.perf_counter() - t0
    cores = min(os.cpu_count() or 1, 16)
    chunks = []
    for e in inst:
        step = max(1, n // max(1, cores // len(inst)))
        chunks += [("C4", _c4_over(*e), lo, min(n, lo + step)) for lo in range(0, n, step)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_sums, chunks)
    dta = time.perf_counter() - t0
    pd = sum(r[2] * r[3] for r in one)
    prices = [(e, _estimate(r[0], r[1], r[2])) for e, r in zip(inst, one)]
    return {"path_dates": pd, "seconds_1core": dt1, "seconds_all": dta, "cores": cores, "prices": prices,
            "paths": n}


def oracle_all_cores(cfg_name, n, over=None):
    """Oracle (price, se, seconds, cores) over paths 0..n-1 in contiguous
    chunks on the host's cores."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    bounds = [(cfg_name, over or {}, i * n // cores, (i + 1) * n // cores) for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_sums, bounds)
    dt = time.perf_counter() - t0
    s = math.fsum(r[0] for r in res)
    ss = math.fsum(r[1] for r in res)
    p, se = _estimate(s, ss, n)
    return p, se, dt, cores, res[0][3]


# -------------------------------------------------------------- workloads ---
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
    lo, hi = S.box_bounds(W.C5_BOX)
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
    steps = (n_train // args.surrogate_batch) * args.surrogate_epochs
    rec["train_step_ms"] = rec["train_s"] / steps * 1e3
    flop_step = 3 * 2.0 * (8 * 256 + 2 * 256 * 256 + 256) * args.surrogate_batch
    rec["train_step_roofline"] = {"bound": "mfma", "achieved": flop_step / (rec["train_step_ms"] * 1e-3) / 1e12,
                                  "peak": 2500.0, "unit": "TFLOP/s (bf16 dense)",
                                  "frac": flop_step / (rec["train_step_ms"] * 1e-3) / 2.5e15}
    rec["train_epochs_batch_lr"] = [args.surrogate_epochs, args.surrogate_batch, args.surrogate_lr]
    rec["train_loss_first_last"] = [losses[0], losses[-1]]
    pred = torch.empty(n_test, dtype=torch.float32, device="cuda")
    sur.infer(torch.tensor(xte, dtype=torch.float32, device="cuda"), pred)
    rec["error_vs_judge"] = S.errors(pred.cpu().numpy(), yte)
    rec["error_plain_mc_2^16_vs_judge"] = S.errors(
        S.mc_prices(pay, xte, c5.n_paths, rate=c5.rate, years_per_day=c5.years_per_day, seed=44)[0], yte)
    nb = c5.notes["infer_batch"]
    xb = torch.tensor(W.c5_points(nb, 45), dtype=torch.float32, device="cuda")
    inf_ms, inf_dev_ms, inf_sync_ms, _ = S.timed_infer(sur, xb)
    rec["infer_batch"] = nb
    rec["infer_ms"] = inf_ms
    rec["infer_device_ms"] = inf_dev_ms
    rec["infer_sync_ms"] = inf_sync_ms
    flop = 2.0 * (8 * 256 + 2 * 256 * 256 + 256) * nb
    rec["infer_roofline"] = {"bound": "mfma", "achieved": flop / (inf_dev_ms * 1e-3) / 1e12, "peak": 2500.0,
                             "unit": "TFLOP/s (bf16 dense)", "frac": flop / (inf_dev_ms * 1e-3) / 2.5e15}
    # the GELU epilogue on the vector unit: 3 x 256 activations per sample,
    # each 5 VALU operations, two transcendentals and half a BF16 pack
    epi_ops = 3 * 256 * 7.5 * nb
    rec["infer_epilogue_roofline"] = {"bound": "alu", "achieved": epi_ops / (inf_dev_ms * 1e-3) / 1e12,
                                      "peak": VALU_PEAK_TOPS, "unit": "T lane-op/s",
                                      "frac": epi_ops / (inf_dev_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS}
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


def hbm_copy_gbs():
    """Device-to-device copy of 1 GiB (read + write bytes per second): the
    HBM bandwidth this machine reaches with a plain copy, beside the 8 TB/s
    published figure."""
    import torch
    src = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 10
    del src, dst
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--quick", action="store_true", help="headline workload only, no CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate workload")
    ap.add_argument("--only", default="",
                    help="comma-separated subset of the extra workloads to run (C1, C2, C2D, C2i, C3, C4sep, "
                         "risk, C5); the headline always runs")
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

    only = set(x.strip() for x in args.only.split(",") if x.strip())
    want = lambda name: not args.quick and (not only or name in only)
    # The oracle's CPU runs go first, before this process touches the GPU
    # (the all-cores runs start worker processes).
    import workloads as W
    cpu = None
    if not args.quick and not args.no_cpu_baseline:
        print("[bench] oracle: C4 sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline_c4()
    oracle_c2 = oracle_c1 = None
    if want("C2") and not args.no_cpu_baseline:
        print("[bench] oracle: C2 at 2^20 Sobol paths", file=sys.stderr, flush=True)
        oracle_c2 = oracle_all_cores("C2", W.C2.n_paths)
    if want("C1") and not args.no_cpu_baseline:
        oracle_c1 = oracle_all_cores("C1", W.C1.n_paths)

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

    # ------------- headline: C4, 1024 templated instances, one graph -------
    c4 = W.C4
    pay4, kw4 = setup(c4)
    T, K, B = W.c4_instances(1024, 42)
    tenv = T.reshape(-1, 1)
    params = np.stack([K, B], 1)
    print("[bench] C4 autotune", file=sys.stderr, flush=True)
    bl, ppt, lanes = P.autotune_batch(pay4, tenv, params, **kw4)
    print(f"[bench] C4 headline at {bl}x{ppt}x{lanes}", file=sys.stderr, flush=True)

    # one complete pmc_price_batch call per step, its arguments marshalled
    # once (the results are read after the timed steps)
    pricer = P.BatchPricer(pay4, tenv, params, **kw4)

    def step():
        return pricer()[0].ms
    # set-up, whatever the warm-up count: the first calls at the tuned tile
    # prepare its tables and capture and instantiate its graph, which later
    # identical calls replay
    step()
    step()
    sec, outs = time_steps(step, args.steps, args.warmup)
    res = pricer.results()
    graph_ms = float(np.mean(outs))
    pd4 = int(sum(r["path_dates"] for r in res))
    value = pd4 / sec
    ops4 = ops_per_path_date(1, "philox", OPS_IL_DOWN_AND_OUT) * pd4
    achieved = ops4 / (graph_ms * 1e-3) / 1e12
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
        "data": "synthetic (seeded Philox streams; instance parameters drawn with numpy default_rng(42))",
        "config": {"workload": "1024 templated down-and-out calls (daily monitoring, 252-1260 dates, strike "
                               "80-120, barrier 50-80% of spot), 2^16 Philox paths each, one persistent "
                               "graph-replayed launch, autotuned tile, FP32 paths, FP64 sums",
                   "instances": 1024, "paths_per_instance": c4.n_paths, "path_dates": pd4,
                   "tile": f"{bl}x{ppt}x{lanes} (threads per block x rounds per thread x paths per lane)",
                   "rng": "philox", "mode": "fused"},
        "device_ms_per_step": graph_ms,
        "engine": "compiled payoff (hipRTC), generic over template environments",
        # graph_ms: HIP events on the library's stream around one graph replay
        # (k_prep, a few microseconds, then the persistent pmc_jit_mc)
        "roofline": {"bound": "alu", "kernel": "pmc_jit_mc<float,philox,1 asset> (persistent, compiled payoff)",
                     "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "T lane-op/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(),
                     "kernel_ms": graph_ms, "algorithmic_ops_per_launch": ops4,
                     "ops_per_path_date": ops_per_path_date(1, "philox", OPS_IL_DOWN_AND_OUT)},
    }
    # error of the headline prices against the oracle: the full-size
    # instances stored by tests/golden/make_oracle_values.py, and the live
    # oracle sample below
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    errs = {}
    if os.path.exists(gpath):
        with open(gpath) as f:
            gfull = json.load(f)["c4_full"]
        if gfull["paths"] == c4.n_paths:
            errs["full_size_stored_oracle"] = {str(e["id"]): err_vs(res[e["id"]]["price"], e["price"], e["se"])
                                               for e in gfull["instances"]}
    if cpu is not None:
        inst, n = cpu["prices"], cpu["paths"]
        ids = np.array([e[0][0] for e in inst], dtype=np.uint32)
        sres = P.price_batch(pay4, np.array([[e[0][1]] for e in inst], np.int32),
                             np.array([[e[0][2], e[0][3]] for e in inst]), instance_ids=ids,
                             **dict(kw4, n_paths=n))
        errs[f"sample_2^{int(math.log2(n))}_paths_live_oracle"] = {
            str(e[0][0]): err_vs(r["price"], e[1][0], e[1][1]) for e, r in zip(inst, sres)}
    allerr = [abs(v["error_in_se"]) for d in errs.values() for v in d.values()]
    line["error_vs_oracle"] = errs
    line["error_vs_oracle_max_se"] = max(allerr) if allerr else None

    extra = {}
    line["hbm_copy_measured_GBs"] = hbm_copy_gbs()
    # measured vector-ALU rates (pmc_probe_valu), beside the derived peak
    probes = {name: ctx.probe_valu(k) / 1e12 for k, name in
              enumerate(("fp32_fma", "int32_xor_add", "mad_u64_u32_add", "fp32_exp2_mul", "fp32_fma_with_xor"))}
    line["valu_measured_T_lane_ops_per_s"] = probes
    line["roofline"]["measured_peak"] = max(probes.values())
    line["roofline"]["frac_of_measured_peak"] = achieved / max(probes.values())
    if want("C4sep"):
        # the same 1024 instruments as separate pmc_price calls
        print("[bench] C4 as 1024 separate calls", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        dev_ms = 0.0
        for i in range(T.size):
            r = P.price(pay4, [int(T[i])], [K[i], B[i]], **dict(kw4, instance=i))
            dev_ms += r["ms"]
            if i % 256 == 255:
                print(f"[bench] C4 separate calls: {i + 1} done", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        extra["C4_separate_pmc_price_calls"] = {"wall_s": wall, "device_ms": dev_ms,
                                                "path_dates_per_s": pd4 / wall,
                                                "graph_replay_speedup_wall": wall / sec}
    if want("C2"):
        # the worst-of autocall, fused, one pmc_price per step
        c2 = W.C2
        pay2, kw2 = setup(c2)
        pricer = P.Pricer(pay2, c2.tenv, c2.params, **kw2)
        s2, t2 = time_steps(lambda: (lambda r: (r.eval_ms, r.ms))(pricer()), 20, 3)
        last = pricer.r.as_dict()
        pd2 = c2.n_paths * last["n_slots"]
        kern_ms = float(np.mean([t[0] for t in t2]))
        il_ops = 3 + (5 * 3 + 4 + 2) / last["n_slots"]
        ops2 = ops_per_path_date(3, "sobol", il_ops) * pd2
        rec = {"ms_per_step": s2 * 1e3, "path_dates_per_s": pd2 / s2, "kernel_ms": kern_ms,
               "device_ms": float(np.mean([t[1] for t in t2])),
               "roofline": {"bound": "alu", "achieved": ops2 / (kern_ms * 1e-3) / 1e12, "peak": VALU_PEAK_TOPS,
                            "unit": "T lane-op/s", "frac": ops2 / (kern_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS},
               "price": last["price"], "std_err": last["std_err"],
               "note": "the Sobol per-wave high-part table is built once per context (k_sobol_hi) and reused "
                       "by every step; it depends only on the path count and dimensions"}
        if oracle_c2 is not None:
            rec["error_vs_oracle"] = err_vs(last["price"], oracle_c2[0], oracle_c2[1])
            rec["oracle_all_cores"] = {"seconds": oracle_c2[2], "cores": oracle_c2[3],
                                       "path_dates_per_s": pd2 / oracle_c2[2]}
        extra["C2_worst_of_autocall"] = rec
        if want("C2i"):
            si, oi = time_steps(lambda: P.price(pay2, c2.tenv, c2.params, engine="interpreter", **kw2), 5, 1)
            extra["C2_interpreter"] = {"ms_per_step": si * 1e3, "path_dates_per_s": pd2 / si,
                                       "kernel_ms": float(np.mean([o["eval_ms"] for o in oi]))}
    if want("C1"):
        # C1: FP64 European call (latency-bound at 2^16 paths), then a sweep
        # to 2^26 paths (2^23 is the paper's vanilla size), each with and
        # without cutPayoff's time guards (Sec. 4.1)
        from oracle.closed_form import bs_call
        c1 = W.C1
        pay1, kw1 = setup(c1)
        s1, o1 = time_steps(lambda: P.price(pay1, c1.tenv, c1.params, **kw1), 20, 3)
        rec = {"ms_per_step": s1 * 1e3, "path_dates_per_s": c1.n_paths / s1,
               "kernel_ms": float(np.mean([o["eval_ms"] for o in o1])),
               "price": o1[-1]["price"], "std_err": o1[-1]["std_err"]}
        if oracle_c1 is not None:
            rec["error_vs_oracle"] = err_vs(o1[-1]["price"], oracle_c1[0], oracle_c1[1])
        extra["C1_fp64_european"] = rec
        ref = bs_call(100.0, 100.0, c1.rate, 0.2, 1.0)
        cut1 = pay1.cut()
        sweep = {}
        for lg in (16, 18, 20, 23, 26):
            kwn = dict(kw1, n_paths=1 << lg)
            sn, on = time_steps(lambda: P.price(pay1, c1.tenv, c1.params, **kwn), 5, 1)
            sc, oc = time_steps(lambda: P.price(cut1, c1.tenv, c1.params, **kwn), 5, 1)
            sweep[f"2^{lg}"] = {"ms_per_step": sn * 1e3, "path_dates_per_s": (1 << lg) / sn,
                                "kernel_ms": float(np.mean([o["eval_ms"] for o in on])),
                                "cut_kernel_ms": float(np.mean([o["eval_ms"] for o in oc])),
                                "cut_ms_per_step": sc * 1e3,
                                "cut_equals_plain": oc[-1]["sum"] == on[-1]["sum"],
                                "error_vs_black_scholes_in_se": (on[-1]["price"] - ref) / on[-1]["std_err"]}
        extra["C1_fp64_european_sweep_with_cut"] = sweep
    if want("C2D"):
        c2d = W.C2D
        pay2d, kw2d = setup(c2d)
        sd, od = time_steps(lambda: P.price(pay2d, c2d.tenv, c2d.params, **kw2d), 20, 3)
        from oracle.closed_form import bs_call
        ref = bs_call(100.0, 100.0, c2d.rate, 0.2, 1.0) + bs_call(100.0, 95.0, c2d.rate, 0.3, 1.0)
        extra["C2D_double_call"] = {"ms_per_step": sd * 1e3, "path_dates_per_s": c2d.n_paths / sd,
                                    "kernel_ms": float(np.mean([o["eval_ms"] for o in od])),
                                    "price": od[-1]["price"], "std_err": od[-1]["std_err"],
                                    "error_vs_black_scholes_sum_in_se": (od[-1]["price"] - ref) / od[-1]["std_err"]}
    if want("C3"):
        # C3: 1260-day down-and-out call, fused and two-phase
        from oracle import closed_form as cf
        c3 = W.C3
        pay3, kw3 = setup(c3)
        bgk = cf.down_and_out_call(100, 100, cf.bgk_barrier(70, 0.3, 1 / 252), 0.03, 0.3, 5.0)
        for mode, engine in (("fused", "compiled"), ("two_phase", "compiled"), ("two_phase", "interpreter")):
            s3, o3 = time_steps(lambda: P.price(pay3, c3.tenv, c3.params, mode=mode, engine=engine, **kw3), 4, 1)
            pd3 = c3.n_paths * o3[-1]["n_slots"]
            rec = {"ms_per_step": s3 * 1e3, "path_dates_per_s": pd3 / s3,
                   "eval_ms": float(np.mean([o["eval_ms"] for o in o3])),
                   "gen_ms": float(np.mean([o["gen_ms"] for o in o3])),
                   "price": o3[-1]["price"], "std_err": o3[-1]["std_err"],
                   "error_vs_bgk_closed_form_in_se": (o3[-1]["price"] - bgk) / o3[-1]["std_err"]}
            if mode == "two_phase":
                # the evaluator reads 4 B per path-date of stored prices
                gbs = 4.0 * pd3 / (rec["eval_ms"] * 1e-3) / 1e9
                rec["eval_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                                        "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
                rec["gen_write_GBs"] = 4.0 * pd3 / (rec["gen_ms"] * 1e-3) / 1e9
            extra[f"C3_down_and_out_{mode}_{engine}"] = rec
    if want("risk"):
        # Risk: delta, gamma and vega of the same 1024 instruments by central
        # differences on common random numbers, 1 + 4A = 5 scenarios each in
        # one persistent launch
        bumps = W.RISK_BUMPS
        sr, orr = time_steps(lambda: P.risk_batch(pay4, tenv, params, **bumps, **kw4), 2, 1)
        n_scen = 1024 * 5
        extra["C4_risk_1024x5"] = {"ms_per_step": sr * 1e3, "pricings_per_s": n_scen / sr,
                                   "greeks_per_s": 3 * 1024 / sr, "path_dates_per_s": 5 * pd4 / sr,
                                   "graph_ms": float(np.mean([r[0]["ms"] for r in orr])),
                                   "bumps": bumps, "instrument_0": orr[-1][0]}
    if want("C5") and not args.no_surrogate:
        extra["C5_surrogate"] = surrogate_workload(ctx, args)
    line["workloads"] = extra

    if cpu is not None:
        line["cpu_baseline"] = {"value": cpu["path_dates"] / cpu["seconds_1core"], "unit": "path-dates/s",
                                "cores": 1, "kind": "oracle",
                                "sample": f"{len(cpu['prices'])} of the 1024 instances (evenly spaced ranks of "
                                          f"their day count), first {cpu['paths']} paths each: "
                                          f"{cpu['path_dates']} path-dates in {cpu['seconds_1core']:.1f} s, "
                                          f"FP64 numpy, one thread",
                                "host": platform.processor() or platform.machine(),
                                "cpu_count": os.cpu_count()}
        line["cpu_oracle_all_cores"] = {"value": cpu["path_dates"] / cpu["seconds_all"], "unit": "path-dates/s",
                                        "cores": cpu["cores"], "seconds": cpu["seconds_all"]}
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
