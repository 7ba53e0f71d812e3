"""GPU parity of the bump-and-revalue risk batch (pmc_risk_batch) against the
oracle's central differences on the same random streams.

Each scenario price is held to the FP32 path bar of the pricing tests
(2e-5 relative to max(1, |V|), continuous payoffs only, so no tie-band);
the Greeks then agree within the bound those price errors allow through the
difference formulas."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import ctx
from oracle import risk as orisk

pytestmark = pytest.mark.gpu

BUMPS = dict(rel_spot_bump=0.01, abs_vol_bump=0.01)


def _check(il, assets, params_lbl, tvars, tenv, params, spot, vol, corr, rng, n, ids=None):
    import paper_2108_03076_amd as P
    pay = P.Payoff(ctx(), il, assets, params_lbl, tvars)
    kw = dict(rate=0.03, years_per_day=1.0 / 252.0)
    I = len(tenv)
    got = P.risk_batch(pay, np.asarray(tenv, np.int32).reshape(I, -1), np.asarray(params).reshape(I, -1),
                       spot=spot, vol=vol, corr=corr, n_paths=n, rng=rng, seed=42, precision="f32",
                       instance_ids=ids, **BUMPS, **kw)
    A = len(assets)
    rel, k = BUMPS["rel_spot_bump"], BUMPS["abs_vol_bump"]
    for i in range(I):
        g = orisk.risk(il, n, spot=spot, vol=vol, rel=rel, k=k, asset_labels=assets, param_labels=params_lbl,
                       params=list(np.asarray(params).reshape(I, -1)[i]),
                       tenv=dict(zip(tvars, np.asarray(tenv).reshape(I, -1)[i].tolist())), corr=corr, rng=rng,
                       seed=42, instance=int(ids[i]) if ids is not None else i, precision="f32", **kw)
        e = [2e-5 * max(1.0, abs(v)) for v in g["scenario_prices"]]
        assert got[i]["price"] == pytest.approx(g["price"], abs=e[0])
        for a in range(A):
            h = rel * spot[a]
            up, dn = 1 + 2 * a, 2 + 2 * a
            assert abs(got[i]["delta"][a] - g["delta"][a]) <= (e[up] + e[dn]) / (2 * h)
            assert abs(got[i]["gamma"][a] - g["gamma"][a]) <= (e[up] + 2 * e[0] + e[dn]) / (h * h)
            vu, vd = 1 + 2 * A + 2 * a, 2 + 2 * A + 2 * a
            assert abs(got[i]["vega"][a] - g["vega"][a]) <= (e[vu] + e[vd]) / (2 * k)
    return got


def test_risk_european_philox():
    print("[risk] european philox", flush=True)
    _check(W.EUROPEAN_CALL, ["S"], ["K"], ["T"], [[252], [126], [504]], [[100.0], [90.0], [115.0]],
           [100.0], [0.2], None, "philox", 3000)


def test_risk_basket_sobol_correlated():
    print("[risk] basket sobol", flush=True)
    corr = W.corr_equi(2, 0.5)
    _check(W.BASKET_CALL, ["S1", "S2"], ["K"], ["T"], [[252], [378]], [[100.0], [105.0]],
           [100.0, 95.0], [0.2, 0.3], corr, "sobol", 2048, ids=np.array([7, 3], np.uint32))


def test_risk_common_random_numbers_forward_gamma():
    """A forward is linear in the spot on every path, so with common random
    numbers its second difference is rounding only; independent streams
    would leave a gamma of order (payoff SD / sqrt(N)) / h^2 ~ 0.5 here."""
    import paper_2108_03076_amd as P
    pay = P.Payoff(ctx(), W.FORWARD, ["S"], ["K"], ["T"])
    g = P.risk_batch(pay, np.array([[252]], np.int32), np.array([[100.0]]), spot=[100.0], vol=[0.25],
                     n_paths=4096, rng="philox", seed=42, precision="f32", rate=0.03,
                     years_per_day=1.0 / 252.0, **BUMPS)[0]
    assert abs(g["gamma"][0]) < 1e-3
    assert g["delta"][0] == pytest.approx(1.0, abs=0.02)


def test_risk_rejects_bad_bumps():
    import paper_2108_03076_amd as P
    pay = P.Payoff(ctx(), W.EUROPEAN_CALL, ["S"], ["K"], ["T"])
    args = (pay, np.array([[252]], np.int32), np.array([[100.0]]))
    kw = dict(spot=[100.0], vol=[0.2], n_paths=256, rng="philox", precision="f32")
    with pytest.raises(P.PmcError):
        P.risk_batch(*args, rel_spot_bump=1.5, abs_vol_bump=0.01, **kw)
    with pytest.raises(P.PmcError):
        P.risk_batch(*args, rel_spot_bump=0.01, abs_vol_bump=0.25, **kw)
