"""The batched launch (templated instances in one persistent, graph-replayed
kernel, Sec. 2 and Sec. 6.2) at the shape the benchmark times: the
1024-instance down-and-out workload with 252..1260 daily dates.

* Sample instances at 2^12 paths, at the tiles (threads per block x rounds
  per thread x paths per lane) 256 x 4 x 1, 128 x 2 x 1 and 128 x 2 x 2
  (two streamed paths per lane) forced through the autotuner's cache file,
  and at the autotuner's own choice: prices against the stored FP64 oracle
  prices on the same streams.
* Exact pins: a vanishing barrier gives the vanilla call on the same
  stream; a barrier at or above the spot knocks out on day 0 (price 0).
* The full batch (1024 x 2^16 paths) at the tuned tile: six instances
  against the stored full-size oracle prices, and properties that hold at
  any size (the down-and-out never exceeds the vanilla on the same paths;
  the vanilla is within its error of Black-Scholes).
* Graph replays follow every launch argument (the seed, the Sobol shape).
"""
import math

import numpy as np
import pytest

import workloads as W
from cases import C4_SAMPLE_PATHS, small
from gpu_common import golden, gpu_payoff, model_kw, opts_kw

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CFG = W.C4


def _sample():
    g = golden()["c4_sample"]
    assert g["paths"] == C4_SAMPLE_PATHS
    inst = g["instances"]
    ids = np.array([e["id"] for e in inst], dtype=np.uint32)
    T = np.array([e["T"] for e in inst], dtype=np.int32).reshape(-1, 1)
    KB = np.array([[e["K"], e["B"]] for e in inst])
    return inst, ids, T, KB


def _tune_key(cache):
    lines = [l.split() for l in cache.read_text().splitlines() if l.strip()]
    assert len(lines) == 1 and len(lines[0]) == 4, lines
    return lines[0][0], int(lines[0][1]), int(lines[0][2]), int(lines[0][3])


def _check_vs_oracle(res, inst, tag):
    """Each price within R18's 0.1 standard errors of the oracle's on the
    same stream; prints the worst case in SE units."""
    worst = 0.0
    for r, e in zip(res, inst):
        d = (r["price"] - e["price"]) / e["se"]
        worst = max(worst, abs(d))
        assert abs(r["price"] - e["price"]) <= 0.1 * e["se"], (tag, e["id"], e["T"], r["price"], e["price"], e["se"])
        assert r["n_slots"] == e["T"] and r["path_dates"] == C4_SAMPLE_PATHS * e["T"]
    print(f"[batch] {tag}: {len(res)} instances, worst |gpu - oracle| = {worst:.4f} SE", flush=True)


def test_sample_instances_at_forced_and_tuned_tiles(tmp_path):
    import paper_2108_03076_amd as P
    inst, ids, T, KB = _sample()
    n = C4_SAMPLE_PATHS
    pay = gpu_payoff(CFG)
    kw = dict(**model_kw(CFG), **opts_kw(CFG, n), instance_ids=ids)
    cache = tmp_path / "tune.txt"
    print("[batch] autotune with a cache file", flush=True)
    bl, pp, ln = P.autotune_batch(pay, T, KB, cache_path=str(cache), **kw)
    key, fbl, fpp, fln = _tune_key(cache)
    assert (fbl, fpp, fln) == (bl, pp, ln) and bl in (64, 128, 256) and pp in (1, 2, 4) and ln in (1, 2)
    tuned = P.price_batch(pay, T, KB, **kw)
    _check_vs_oracle(tuned, inst, f"tuned {bl}x{pp}x{ln}")
    results = {}
    for tile in ((256, 4, 1), (128, 2, 1), (128, 2, 2)):
        cache.write_text(f"{key} {tile[0]} {tile[1]} {tile[2]}\n")
        assert P.autotune_batch(pay, T, KB, cache_path=str(cache), **kw) == tile
        print(f"[batch] forced tile {tile}", flush=True)
        res = P.price_batch(pay, T, KB, **kw)
        _check_vs_oracle(res, inst, f"tile {tile}")
        results[tile] = res
    # the same paths whatever the tile: sums agree up to their order
    for t in ((128, 2, 1), (128, 2, 2)):
        for a, b in zip(results[(256, 4, 1)], results[t]):
            assert a["sum"] == pytest.approx(b["sum"], rel=1e-12, abs=1e-9), t
    # a cache entry that is not a launchable tile is ignored (tuned again)
    for bad in ("100 0 1", "128 2 3"):
        cache.write_text(f"{key} {bad}\n")
        bl2, pp2, ln2 = P.autotune_batch(pay, T, KB, cache_path=str(cache), **kw)
        assert bl2 % 64 == 0 and 64 <= bl2 <= 256 and pp2 >= 1 and ln2 in (1, 2)


def test_sample_instances_equal_single_prices():
    """Each batch instance prices the same paths as a single pmc_price call
    with that instance's counter word."""
    import paper_2108_03076_amd as P
    inst, ids, T, KB = _sample()
    n = C4_SAMPLE_PATHS
    pay = gpu_payoff(CFG)
    res = P.price_batch(pay, T, KB, **model_kw(CFG), **opts_kw(CFG, n), instance_ids=ids)
    for i in (0, len(inst) // 2, len(inst) - 1):
        one = P.price(pay, [int(T[i, 0])], list(KB[i]), **model_kw(CFG), **opts_kw(CFG, n, instance=int(ids[i])))
        assert res[i]["sum"] == pytest.approx(one["sum"], rel=1e-12, abs=1e-9), i


def test_barrier_pins():
    import paper_2108_03076_amd as P
    inst, ids, T, KB = _sample()
    n = C4_SAMPLE_PATHS
    pay = gpu_payoff(CFG)
    kw = dict(**model_kw(CFG), **opts_kw(CFG, n), instance_ids=ids)
    # barrier 0: never hit (prices are positive), so the vanilla call on the
    # same paths, which the oracle side writes without the IL
    van = P.price_batch(pay, T, np.stack([KB[:, 0], np.zeros(len(inst))], 1), **kw)
    worst = 0.0
    for r, e in zip(van, inst):
        worst = max(worst, abs(r["price"] - e["vanilla_price"]) / e["vanilla_se"])
        assert abs(r["price"] - e["vanilla_price"]) <= 0.1 * e["vanilla_se"], (e["id"], r["price"], e)
    print(f"[batch] vanishing barrier: worst |gpu - vanilla| = {worst:.4f} SE", flush=True)
    # barrier at or above the spot: knocked out on day 0, exactly zero
    for b in (100.0, 150.0):
        out = P.price_batch(pay, T, np.stack([KB[:, 0], np.full(len(inst), b)], 1), **kw)
        assert all(r["price"] == 0.0 and r["std_err"] == 0.0 for r in out)


def test_full_batch_at_tuned_tile():
    import paper_2108_03076_amd as P
    from oracle.closed_form import bs_call
    g = golden()["c4_full"]
    n = CFG.n_paths
    assert g["paths"] == n
    T, K, B = W.c4_instances(1024, 42)
    tenv = T.reshape(-1, 1)
    pay = gpu_payoff(CFG)
    kw = dict(**model_kw(CFG), **opts_kw(CFG, n))
    bl, pp, ln = P.autotune_batch(pay, tenv, np.stack([K, B], 1), **kw)
    print(f"[batch] full 1024 x 2^16 at {bl}x{pp}x{ln}", flush=True)
    do = P.price_batch(pay, tenv, np.stack([K, B], 1), **kw)
    van = P.price_batch(pay, tenv, np.stack([K, np.zeros_like(B)], 1), **kw)
    worst = 0.0
    for e in g["instances"]:
        r = do[e["id"]]
        assert (int(T[e["id"]]), K[e["id"]], B[e["id"]]) == (e["T"], e["K"], e["B"])
        worst = max(worst, abs(r["price"] - e["price"]) / e["se"])
        assert abs(r["price"] - e["price"]) <= 0.1 * e["se"], (e["id"], r["price"], e)
    print(f"[batch] full size: worst |gpu - oracle| = {worst:.4f} SE over {len(g['instances'])} instances",
          flush=True)
    z = []
    for i in range(T.size):
        # per path the knock-out payoff is at most the vanilla one; the two
        # batches sum their paths in the same order, and rounded addition is
        # monotone, so the sums keep the order
        assert do[i]["sum"] <= van[i]["sum"], i
        ref = bs_call(100.0, K[i], CFG.rate, 0.2, T[i] / 252.0)
        z.append((van[i]["price"] - ref) / van[i]["std_err"])
    z = np.array(z)
    print(f"[batch] vanilla vs Black-Scholes: max |z| {np.abs(z).max():.2f}, mean z {z.mean():.3f}", flush=True)
    # 1024 instances: |z| > 4.5 has probability 7e-6 each
    assert np.abs(z).max() < 4.5
    assert abs(z.mean()) < 4.5 / math.sqrt(T.size)


def test_batch_graph_replays_follow_the_seed():
    """A batch graph captured for one seed is not replayed for another seed
    of the same shape (the Philox key is a by-value kernel argument)."""
    import paper_2108_03076_amd as P
    cfg = small(CFG)
    T = np.array([[20], [45], [7], [33], [60], [1], [0], [52]], dtype=np.int32)
    KB = np.stack([np.linspace(90, 110, 8), np.linspace(60, 95, 8)], 1)
    n = 2048
    pay = gpu_payoff(cfg)
    res = {}
    for seed in (42, 7, 42):
        out = P.price_batch(pay, T, KB, **model_kw(cfg), **opts_kw(cfg, n, seed=seed))
        for i in range(len(T)):
            one = P.price(pay, [int(T[i, 0])], list(KB[i]), **model_kw(cfg), **opts_kw(cfg, n, seed=seed, instance=i))
            assert out[i]["sum"] == pytest.approx(one["sum"], rel=1e-12, abs=1e-9), (seed, i)
        if seed in res:
            assert [r["sum"] for r in out] == [r["sum"] for r in res[seed]]
        res[seed] = out
    assert any(a["sum"] != b["sum"] for a, b in zip(res[42], res[7]) if a["n_slots"] > 0)


def test_batch_graph_replays_follow_the_sobol_shape():
    """Sobol batches of fewer paths than one tile keep the same grid but not
    the same number of Gray-code bits."""
    import paper_2108_03076_amd as P
    cfg = W.C2
    tenv = np.array([[4], [4]], dtype=np.int32)
    pay = gpu_payoff(cfg)
    for n in (100, 200, 100):
        out = P.price_batch(pay, tenv, np.zeros((2, 0)), **model_kw(cfg), **opts_kw(cfg, n))
        one = P.price(pay, cfg.tenv, [], **model_kw(cfg), **opts_kw(cfg, n))
        assert out[0]["sum"] == pytest.approx(one["sum"], rel=1e-12), n


def test_untuned_tiles_price_the_same_paths(tmp_path):
    """Without an autotuned tile a batch picks its own: two streamed paths
    per lane for the down-and-out sample, and for the short paths of the
    surrogate's worst-of family (3 assets, 1-5 dates, a model per point)
    more paths per thread than the item count alone asks for.  Either way
    each instance prices the same paths as at a forced one-path tile: the
    sums agree up to their order.  (Fresh contexts: no tuned entry leaks
    into the other tests.)"""
    import paper_2108_03076_amd as P
    from paper_2108_03076_amd import surrogate as S
    inst, ids, T, KB = _sample()
    c5 = W.C5
    pts = W.c5_points(64, 77)
    fb = S.family_batch(pts)
    cases = [
        ("down-and-out", CFG, T, KB, dict(**model_kw(CFG), **opts_kw(CFG, C4_SAMPLE_PATHS), instance_ids=ids)),
        ("worst-of family", c5, fb["tenv"], fb["params"],
         dict(spot=fb["spot"], vol=fb["vol"], corr=fb["corr"], per_instance_model=True, rate=c5.rate,
              years_per_day=c5.years_per_day, n_paths=1 << 14, rng="philox", seed=42, precision="f32",
              instance_ids=np.arange(64, dtype=np.uint32))),
    ]

    def payoff(cfg):
        return P.Payoff(P.Context(0), cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)

    for name, cfg, tenv, params, kw in cases:
        print(f"[batch] untuned tile: {name}", flush=True)
        untuned = P.price_batch(payoff(cfg), tenv, params, **kw)
        cache = tmp_path / (name.replace(" ", "_") + ".txt")
        P.autotune_batch(payoff(cfg), tenv, params, cache_path=str(cache), **kw)
        key = _tune_key(cache)[0]
        cache.write_text(f"{key} 256 1 1\n")
        pay = payoff(cfg)
        assert P.autotune_batch(pay, tenv, params, cache_path=str(cache), **kw) == (256, 1, 1)
        forced = P.price_batch(pay, tenv, params, **kw)
        for a, b in zip(untuned, forced):
            assert a["path_dates"] == b["path_dates"]
            assert a["sum"] == pytest.approx(b["sum"], rel=1e-12, abs=1e-9), name


def test_batch_pricer_equals_price_batch():
    """The prepared batch call (arguments marshalled once, for timing loops)
    returns what price_batch returns, call after call."""
    import paper_2108_03076_amd as P
    inst, ids, T, KB = _sample()
    pay = gpu_payoff(CFG)
    kw = dict(**model_kw(CFG), **opts_kw(CFG, C4_SAMPLE_PATHS), instance_ids=ids)
    ref = P.price_batch(pay, T, KB, **kw)
    pricer = P.BatchPricer(pay, T, KB, **kw)
    for _ in range(3):
        pricer()
        got = pricer.results()
        assert [(r["sum"], r["sum_sq"], r["path_dates"]) for r in got] == \
            [(r["sum"], r["sum_sq"], r["path_dates"]) for r in ref]
