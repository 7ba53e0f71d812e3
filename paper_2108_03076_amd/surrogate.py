"""Learned surrogate workflow on top of the C ABI: label generation by the
batched Monte Carlo engine, training and inference by the library's MLP
kernels, and the Monte Carlo judge of the surrogate's error.

The surrogate maps (3 spots, 3 vols, pairwise correlation, number of annual
observation dates) to the price of the worst-of autocall family; the number
of dates n maps to the template variable N = n - 1 of the payoff expression,
and each point's model (spots, vols, equicorrelation) is a per-instance
model of one batched launch.  Every number is computed on the GPU; this
module only orders the calls.
"""
from __future__ import annotations

import time

import numpy as np

from ._lib import Context, Payoff, Surrogate, price_batch


def equicorr(rho):
    """[n][3][3] equicorrelation matrices."""
    rho = np.asarray(rho, dtype=np.float64).reshape(-1)
    c = np.repeat(np.eye(3)[None], rho.size, axis=0)
    for i in range(3):
        for j in range(3):
            if i != j:
                c[:, i, j] = rho
    return c


def box_bounds(box):
    """Per-input (lo, hi) of the surrogate's box: 3 spots, 3 vols, the
    pairwise correlation and the number of dates."""
    lo = [box["spot"][0]] * 3 + [box["vol"][0]] * 3 + [box["rho"][0], box["n_obs"][0]]
    hi = [box["spot"][1]] * 3 + [box["vol"][1]] * 3 + [box["rho"][1], box["n_obs"][1]]
    return lo, hi


def mc_prices(pay: Payoff, points, n_paths, *, rate, years_per_day, seed, first_id=0, chunk=1 << 15,
              engine="auto"):
    """Monte Carlo prices (and standard errors) of the points [n][8] with one
    batched launch per chunk of points; point i uses Philox counter word 2 =
    first_id + i."""
    pts = np.asarray(points, dtype=np.float64)
    n = pts.shape[0]
    price = np.zeros(n)
    se = np.zeros(n)
    path_dates = 0
    gpu_ms = 0.0
    for o in range(0, n, chunk):
        p = pts[o:o + chunk]
        k = p.shape[0]
        tenv = (p[:, 7].astype(np.int32) - 1).reshape(-1, 1)
        res = price_batch(pay, tenv, np.zeros((k, 0)), spot=p[:, 0:3], vol=p[:, 3:6], corr=equicorr(p[:, 6]),
                          rate=rate, years_per_day=years_per_day, per_instance_model=True,
                          instance_ids=np.arange(first_id + o, first_id + o + k, dtype=np.uint32),
                          n_paths=n_paths, rng="philox", seed=seed, precision="f32", engine=engine)
        price[o:o + k] = [r["price"] for r in res]
        se[o:o + k] = [r["std_err"] for r in res]
        path_dates += sum(r["path_dates"] for r in res)
        gpu_ms += res[0]["ms"]
    return price, se, path_dates, gpu_ms


def family_batch(points):
    """The worst-of autocall instances of points [n][8]: template variable
    N = n_obs - 1 and a per-point model (spots, vols, equicorrelation)."""
    p = np.asarray(points, dtype=np.float64)
    tenv = (np.rint(p[:, 7]).astype(np.int32) - 1).reshape(-1, 1)
    return dict(tenv=tenv, params=np.zeros((p.shape[0], 0)), spot=p[:, 0:3], vol=p[:, 3:6],
                corr=equicorr(p[:, 6]), per_instance_model=True)


def price_with_fallback(sur: Surrogate, pay: Payoff, points, n_paths, *, rate, years_per_day, seed, first_id=0):
    """Prices of points [n][8]: the surrogate inside its input box, the
    batched Monte Carlo engine (n_paths Philox paths, point i on stream
    first_id + i) outside it (pmc_mlp_price).  Returns (price, Monte Carlo
    standard error or 0, route: 0 surrogate, 1 Monte Carlo)."""
    p = np.asarray(points, dtype=np.float64)
    ids = np.arange(first_id, first_id + p.shape[0], dtype=np.uint32)
    return sur.price(p, pay, **family_batch(p), rate=rate, years_per_day=years_per_day, instance_ids=ids,
                     n_paths=n_paths, rng="philox", seed=seed, precision="f32")


def train(sur: Surrogate, x, y, *, epochs, batch=4096, lr_max=1e-3, lr_min=1e-5, log=None):
    """Trains on device tensors x [n][8] (float32) and y [n] (float32) with a
    cosine learning-rate schedule over all steps; returns per-epoch losses."""
    import torch
    n = int(y.numel())
    steps = max(1, n // batch) * epochs
    losses = []
    # the shuffle runs on the device (on torch's current stream, which a
    # context uses unless given another)
    g = torch.Generator(device=x.device).manual_seed(0)
    for e in range(epochs):
        perm = torch.randperm(n, generator=g, device=x.device)
        xe, ye = x[perm].contiguous(), y[perm].contiguous()
        losses.append(sur.train_epoch(xe, ye, batch=batch, lr_max=lr_max, lr_min=lr_min, total_steps=steps))
        if log:
            log(f"epoch {e} loss {losses[-1]:.3e}")
    return losses


def errors(pred, ref):
    """RMS, 99th percentile and max of |pred - ref| / |ref|."""
    rel = np.abs(np.asarray(pred, np.float64) - ref) / np.abs(ref)
    return {"rms": float(np.sqrt(np.mean(rel * rel))), "p99": float(np.quantile(rel, 0.99)),
            "max": float(rel.max())}


def timed_infer(sur: Surrogate, x, reps=20):
    """Inference over the rows of x, timed three ways (ms per call): calls
    issued back to back (the call is stream-ordered, so this is the rate a
    serving loop sees), the device time between events bracketing single
    calls on the context's stream (torch's current stream, which the
    surrogate launches on), and a call followed by a synchronization (the
    latency of one isolated request).  Returns (pipelined, device,
    synchronous, predictions)."""
    import torch
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    sur.infer(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sur.infer(x, y)
    torch.cuda.synchronize()
    pipelined = (time.perf_counter() - t0) / reps * 1e3
    dev = 0.0
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sur.infer(x, y)
        b.record()
        b.synchronize()
        dev += a.elapsed_time(b)
    sync = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        sur.infer(x, y)
        torch.cuda.synchronize()
        sync += time.perf_counter() - t0
    return pipelined, dev / reps, sync / reps * 1e3, y


__all__ = ["box_bounds", "equicorr", "family_batch", "price_with_fallback", "mc_prices", "train", "errors", "timed_infer", "Context", "Surrogate"]
