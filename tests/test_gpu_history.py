"""Pricing at a current day on a caller-supplied price history (Sec. 4.1:
the environment is historical data up to the current time and simulated
data after it; Thm. 5 for the cut payoff), through the C ABI against the
FP64 oracle on the same random streams: the simulation starts on the
current day from the history's last prices, history days (before the
history's first day: its first price) are read from the history.

Bars (R18): FP64 prices within 1e-12 relative; FP32 prices within 0.1
standard errors plus the per-path FP32 bar of 1e-5 relative (a price that
the history alone fixes has no standard error, and its history prices are
rounded to FP32 on the device); a history that knocks the contract out
prices exactly 0; generated paths within 2e-5 relative of the oracle's on
every slot."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from gpu_common import gpu_payoff, model_kw, opts_kw, oracle_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _walk(n, seed, start=100.0, vol=0.01):
    g = np.random.default_rng(seed)
    return start * np.exp(vol * np.cumsum(g.normal(size=n)))


def _check(cfg, pay_il, hist, now, n, tag, **opts):
    import paper_2108_03076_amd as P
    from oracle.il import cut_payoff, parse
    from oracle.mc import estimate
    pay = gpu_payoff(cfg, il=pay_il)
    cut = pay.cut()
    prob = oracle_problem(cfg, il=cut_payoff(parse(pay_il)), t_now=now, history=hist)
    ref, se = estimate(prob.payoffs(np.arange(n)))
    r = P.price(cut, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n, t_now=now, history=hist, **opts))
    print(f"[history] {tag} now={now}: gpu {r['price']:.8f} oracle {ref:.8f} se {se:.5f} slots {r['n_slots']}",
          flush=True)
    assert r["n_slots"] == len(prob.days)
    if cfg.precision == "f64":
        assert r["price"] == pytest.approx(ref, rel=1e-12, abs=1e-12), (tag, now)
    else:
        assert abs(r["price"] - ref) <= 0.1 * se + 1e-5 * max(1.0, abs(ref)), (tag, now, r["price"], ref, se)
    return r, ref


@pytest.mark.parametrize("engine", ["interpreter", "compiled"])
@pytest.mark.parametrize("mode", ["fused", "two_phase"])
def test_down_and_out_on_history(engine, mode):
    cfg = dataclasses.replace(W.C3, tenv=[60])
    for now in (0, 1, 37, 60, 75):
        hist = [_walk(now + 3, now)]          # days now-2 .. now, above the barrier
        assert hist[0].min() > 70.0
        _check(cfg, cfg.il, hist, now, 3000, f"down-and-out {engine} {mode}", engine=engine, mode=mode)
    # a history touching the barrier: every path is knocked out
    hit = _walk(41, 1)
    hit[5] = 65.0
    r, ref = _check(cfg, cfg.il, [hit], 40, 1024, f"knocked out {engine} {mode}", engine=engine, mode=mode)
    assert r["price"] == 0.0 and ref == 0.0


@pytest.mark.parametrize("engine", ["interpreter", "compiled"])
def test_european_fp64_and_worst_of_on_history(engine):
    c1 = W.C1
    _check(c1, c1.il, [[95.0, 104.0, 110.0]], 100, 4096, f"european fp64 {engine}", engine=engine)
    c2 = W.C2
    hist = [_walk(2, 11), _walk(2, 12), _walk(2, 13)]   # days 1 and 2; earlier days read day 1
    for now in (2, 4):
        h = [np.concatenate([x, _walk(now - 2, 20 + a, start=x[-1])]) for a, x in enumerate(hist)]
        _check(c2, c2.il, h, now, 2048, f"worst-of sobol {engine}", engine=engine)


def test_batch_and_paths_on_history():
    """A batch of instances on one history gives their single prices (the
    same per-path payoffs, summed in another order: 1e-12 relative);
    generated paths start from the history's last price."""
    import paper_2108_03076_amd as P
    cfg = dataclasses.replace(W.C3, tenv=[60])
    now = 25
    hist = [_walk(now + 1, 3)]
    pay = gpu_payoff(cfg).cut()
    T = np.array([[40], [60], [90]], dtype=np.int32)
    KB = np.array([[95.0, 70.0], [100.0, 72.0], [105.0, 68.0]])
    res = P.price_batch(pay, T, KB, **model_kw(cfg), **opts_kw(cfg, 4096, t_now=now, history=hist))
    for i in range(3):
        one = P.price(pay, T[i], KB[i], **model_kw(cfg), **opts_kw(cfg, 4096, t_now=now, history=hist, instance=i,
                                                               mode="fused"))
        print(f"[history] batch instance {i}: {res[i]['price']:.6f} single {one['price']:.6f}", flush=True)
        assert res[i]["n_slots"] == one["n_slots"] == int(T[i][0]) - now
        assert abs(res[i]["price"] - one["price"]) <= 1e-12 * max(1.0, abs(one["price"]))
    n = 2048
    prob = oracle_problem(cfg, t_now=now, history=hist)
    S = torch.zeros((len(prob.days), 1, n), dtype=torch.float32, device="cuda")
    P.gen_paths(gpu_payoff(cfg), S, tenv=cfg.tenv, **model_kw(cfg), **opts_kw(cfg, n, t_now=now, history=hist))
    got = S.cpu().numpy().astype(np.float64).transpose(2, 0, 1)
    ref = prob.paths(np.arange(n))
    assert np.max(np.abs(got - ref) / ref) <= 2e-5
    rel0 = np.abs(ref[:, 0, 0] / hist[0][-1] - 1)
    assert rel0.max() < 0.1     # one day from the history's last price
