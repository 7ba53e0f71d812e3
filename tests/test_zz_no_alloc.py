"""pmc_price_noalloc, the allocation-free pricing call, through the C ABI:
two calls in a row (the second on a smaller input) against pmc_price by the
same engine and mode (bit-identical sums and per-path payoffs), the smaller
call also against the FP64 oracle on the same stream (0.1 standard errors in
FP32, 1e-12 relative in FP64), and its documented refusals."""
import numpy as np
import pytest

import workloads as W
from gpu_common import ctx, gpu_payoff, model_kw, oracle_problem, opts_kw

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(pay, cfg, tenv, n):
    """(pmc_price, pmc_price_noalloc) results and per-path payoffs."""
    import paper_2108_03076_amd as P
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    ya = torch.full((n,), float("nan"), dtype=dt, device="cuda")
    yb = torch.full((n,), float("nan"), dtype=dt, device="cuda")
    kw = dict(engine="interpreter", mode="fused")
    a = P.price(pay, tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n, payoffs=ya, **kw))
    b = P.price_noalloc(pay, tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n, payoffs=yb))
    torch.cuda.synchronize()
    return a, b, ya.cpu().numpy(), yb.cpu().numpy()


CASES = [
    # (workload, template environment, first paths, second (smaller) tenv and paths)
    ("c2_sobol_3_assets", W.C2, [4], 16421, [2], 1000),
    ("c3_down_and_out", W.C3, [300], 50000, [60], 3001),
    ("c1_fp64", W.C1, [252], 1 << 16, [126], 777),
]


@pytest.mark.parametrize("name,cfg,tenv1,n1,tenv2,n2", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_price_on_two_calls(name, cfg, tenv1, n1, tenv2, n2):
    pay = gpu_payoff(cfg)
    for tenv, n in ((tenv1, n1), (tenv2, n2)):
        print(f"[noalloc] {name}: tenv {tenv}, {n} paths", flush=True)
        a, b, ya, yb = _pair(pay, cfg, tenv, n)
        assert (b["sum"], b["sum_sq"]) == (a["sum"], a["sum_sq"]), (name, tenv, n, a, b)
        assert b["n_paths"] == n and b["n_slots"] == a["n_slots"] and b["path_dates"] == a["path_dates"]
        assert b["engine_used"] == 1 and b["mode_used"] == 2
        assert np.array_equal(ya, yb), (name, tenv, n)
    # the smaller call against the oracle on the same stream
    prob = oracle_problem(cfg, tenv=dict(zip(cfg.tvars, tenv2)))
    ref = prob.payoffs(np.arange(n2))
    p, se = float(np.mean(ref)), float(np.std(ref, ddof=1) / np.sqrt(n2))
    tol = 1e-12 * abs(p) if cfg.precision == "f64" else 0.1 * se
    print(f"[noalloc] {name}: gpu {b['price']:.8f} oracle {p:.8f} se {se:.5f}", flush=True)
    assert abs(b["price"] - p) <= tol, (name, b["price"], p, se)


def test_noalloc_refusals_leave_later_calls_working():
    import paper_2108_03076_amd as P
    cfg = W.C2
    pay = gpu_payoff(cfg)
    for over in ({"mode": "two_phase"}, {"engine": "compiled"}):
        with pytest.raises(P.PmcError) as e:
            P.price_noalloc(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, 1024, **over))
        assert e.value.name == "E_UNSUPPORTED", over
    # 3 assets x 6000 daily dates: 18000 Sobol dimensions, whose direction
    # numbers alone exceed the scratch's 2 MiB table area
    il = "(loopif (leq (model S1 0) (real 0.0)) (real 0.0) (payoff 0 X Y) 6000)"
    big = P.Payoff(ctx(), il, ["S1", "S2", "S3"], [], [])
    with pytest.raises(P.PmcError) as e:
        P.price_noalloc(big, [], [], **model_kw(cfg), **opts_kw(cfg, 1024))
    assert e.value.name == "E_UNSUPPORTED" and "scratch" in str(e.value)
    print("[noalloc] refusals:", str(e.value), flush=True)
    a, b, ya, yb = _pair(pay, cfg, cfg.tenv, 2048)
    assert (b["sum"], b["sum_sq"]) == (a["sum"], a["sum_sq"])
