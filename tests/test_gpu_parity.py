"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded streams.

Bars (FP32 paths): random words bit-exact; normals within 2e-6 (AS241's
7-digit variant in binary32 against PPND16 in binary64); prices on every
simulated day within 2e-5 relative (binary32 log-price accumulation over up
to 1260 steps); per-path payoffs within 1e-5 relative outside the tie-band
(paths whose oracle payoff jumps when every price moves by 3e-5);
prices within 0.1 standard errors.  FP64 paths: normals and prices within
1e-13 relative, prices within 1e-12 relative.
"""
import math

import numpy as np
import pytest

import workloads as W
from cases import PARITY, small as _small
from gpu_common import check_band, golden, gpu_payoff, model_kw, opts_kw, oracle_problem, sample_ids, tie_band

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gen(cfg, n, tenv=None):
    import paper_2108_03076_amd as P
    tenv = cfg.tenv if tenv is None else tenv
    pay = gpu_payoff(cfg)
    days, _ = pay.grid(tenv)
    A = len(cfg.asset_labels)
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    paths = torch.empty(len(days) * A * n, dtype=dt, device="cuda")
    words = torch.empty(len(days) * A * n, dtype=torch.int32, device="cuda")
    normals = torch.empty(len(days) * A * n, dtype=dt, device="cuda")
    P.gen_paths(pay, paths, words, normals, tenv, **model_kw(cfg), **opts_kw(cfg, n))
    torch.cuda.synchronize()
    D = len(days)
    S = paths.double().cpu().numpy().reshape(D, A, n).transpose(2, 0, 1)          # [path][slot][asset]
    wd = words.cpu().numpy().view(np.uint32).reshape(D * A, n).T                  # [path][word]
    z = normals.double().cpu().numpy().reshape(D * A, n).T
    return pay, days, S, wd, z, paths


CASES = PARITY


@pytest.mark.parametrize("name", list(CASES))
def test_streams_and_paths(name):
    cfg = CASES[name]
    n = 1000                                     # ragged: 3 full blocks of 256 and a tail
    print(f"[parity] streams {name} n={n}", flush=True)
    pay, days, S, wd, z, _ = _gen(cfg, n)
    prob = oracle_problem(cfg)
    assert days == prob.days
    ids = np.arange(n)
    ow = prob.words(ids)
    assert np.array_equal(wd, ow), "random words differ"
    oz = prob.normals(ids).reshape(n, -1)
    oS = prob.paths(ids)
    if cfg.precision == "f64":
        assert np.max(np.abs(z - oz) / np.maximum(1, np.abs(oz))) < 1e-13
        assert np.max(np.abs(S / oS - 1)) < 1e-13
    else:
        assert np.max(np.abs(z - oz) / np.maximum(1, np.abs(oz))) < 2e-6
        assert np.max(np.abs(S / oS - 1)) < 2e-5


# Philox cases for the path store's block-ordered loop: 1 asset (37 slots: a
# ragged group; 1 slot: the ragged group alone), 2 assets (groups of 2
# slots), 3 assets (5 slots: one group of 4 and one slot; 12 slots: whole
# groups only), FP32 and FP64.
_PHILOX_STORE = {
    "c3_short": CASES["c3_short"],
    "c1": CASES["c1"],
    "c2_philox": CASES["c2_philox"],
    "c2d_philox": _small(CASES["c2d"], rng="philox"),
    "c2_long_philox": _small(CASES["c2_long"], rng="philox"),
    "c2_f64_philox": _small(CASES["c2_f64"], rng="philox"),
}


@pytest.mark.parametrize("name", list(_PHILOX_STORE))
@pytest.mark.parametrize("n", [1000, 64])
def test_path_store_without_recording_equals_recorded(name, n):
    """Generating the path store alone (no words or normals recorded) takes
    the Philox blocks in counter order; its prices equal, bit for bit, the
    ones generated while recording, which test_streams_and_paths compares
    with the oracle."""
    import paper_2108_03076_amd as P
    cfg = _PHILOX_STORE[name]
    print(f"[parity] path store {name} n={n}", flush=True)
    pay = gpu_payoff(cfg)
    days, _ = pay.grid(cfg.tenv)
    A = len(cfg.asset_labels)
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    rec = torch.empty(len(days) * A * n, dtype=dt, device="cuda")
    words = torch.empty(len(days) * A * n, dtype=torch.int32, device="cuda")
    normals = torch.empty(len(days) * A * n, dtype=dt, device="cuda")
    P.gen_paths(pay, rec, words, normals, cfg.tenv, **model_kw(cfg), **opts_kw(cfg, n))
    alone = torch.full_like(rec, float("nan"))
    P.gen_paths(pay, alone, None, None, cfg.tenv, **model_kw(cfg), **opts_kw(cfg, n))
    torch.cuda.synchronize()
    assert torch.equal(alone, rec)
    S = alone.double().cpu().numpy().reshape(len(days), A, n).transpose(2, 0, 1)
    oS = oracle_problem(cfg).paths(np.arange(n))
    tol = 1e-13 if cfg.precision == "f64" else 2e-5
    assert np.max(np.abs(S / oS - 1)) < tol


@pytest.mark.parametrize("name", list(CASES))
def test_payoffs_on_stored_paths(name):
    """Payoff arithmetic alone: the GPU evaluates its own stored paths, the
    oracle evaluates the same values upcast exactly to binary64."""
    import paper_2108_03076_amd as P
    cfg = CASES[name]
    n = 1000
    print(f"[parity] eval_paths {name}", flush=True)
    pay, days, S, _, _, paths = _gen(cfg, n)
    prob = oracle_problem(cfg)
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    out = torch.empty(n, dtype=dt, device="cuda")
    r = P.eval_paths(pay, paths, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n, payoffs=out))
    gpu = out.double().cpu().numpy()
    ref = prob.payoffs_on_paths(S)
    tol = 1e-12 if cfg.precision == "f64" else 1e-5
    band = tie_band(prob, S, 3e-5) if cfg.precision == "f32" else np.zeros(n, bool)
    if cfg.precision == "f32":
        check_band(f"parity/{name}", band)
    bad = (np.abs(gpu - ref) > tol * np.maximum(np.abs(ref), 1.0)) & ~band
    assert not bad.any(), (np.nonzero(bad)[0][:10], gpu[bad][:5], ref[bad][:5])
    assert r["sum"] == pytest.approx(gpu.sum(), rel=1e-12, abs=1e-9)


@pytest.mark.parametrize("name", ["c3_short", "c2", "c1"])
@pytest.mark.parametrize("n,offset", [(1028, 0), (1001, 0), (4, 0), (1000, 1)])
def test_stored_paths_lane_layouts(name, n, offset):
    """The compiled evaluator of stored paths takes 4 (FP32) or 2 (FP64)
    paths per lane when the path count and the buffer alignment allow it and
    one otherwise (a count not a multiple of 4, a buffer one element off);
    every layout gives the interpreter's per-path payoffs exactly."""
    import paper_2108_03076_amd as P
    cfg = CASES[name]
    print(f"[parity] lanes {name} n={n} offset={offset}", flush=True)
    pay, days, S, _, _, paths = _gen(cfg, n)
    if offset:
        big = torch.empty(paths.numel() + offset, dtype=paths.dtype, device="cuda")
        big[offset:].copy_(paths)
        paths = big[offset:]
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    outs = {}
    for engine in ("interpreter", "compiled"):
        out = torch.empty(n, dtype=dt, device="cuda")
        r = P.eval_paths(pay, paths, cfg.tenv, cfg.params, **model_kw(cfg),
                         **opts_kw(cfg, n, payoffs=out, engine=engine))
        outs[engine] = (out.cpu(), r)
    assert torch.equal(outs["interpreter"][0], outs["compiled"][0])
    ref = oracle_problem(cfg).payoffs_on_paths(S)
    gpu = outs["compiled"][0].double().numpy()
    tol = 1e-12 if cfg.precision == "f64" else 1e-5
    band = tie_band(oracle_problem(cfg), S, 3e-5) if cfg.precision == "f32" else np.zeros(n, bool)
    if cfg.precision == "f32":
        check_band(f"parity/{name}", band)
    assert not ((np.abs(gpu - ref) > tol * np.maximum(np.abs(ref), 1.0)) & ~band).any()
    assert outs["compiled"][1]["sum"] == pytest.approx(gpu.sum(), rel=1e-12, abs=1e-9)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mode", ["fused", "two_phase"])
@pytest.mark.parametrize("engine", ["interpreter", "compiled"])
def test_price_matches_oracle(name, mode, engine):
    import paper_2108_03076_amd as P
    cfg = CASES[name]
    n = 4000 if cfg.precision == "f32" else 1 << 14
    print(f"[parity] price {name} {mode} {engine} n={n}", flush=True)
    pay = gpu_payoff(cfg)
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    out = torch.empty(n, dtype=dt, device="cuda")
    r = P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg),
                **opts_kw(cfg, n, mode=mode, payoffs=out, engine=engine))
    assert r["engine_used"] == (1 if engine == "interpreter" else 2)
    prob = oracle_problem(cfg)
    ids = np.arange(n)
    ref_pay = prob.payoffs(ids)
    from oracle.mc import estimate
    ref, se = estimate(ref_pay)
    gpu = out.double().cpu().numpy()
    if cfg.precision == "f64":
        assert r["price"] == pytest.approx(ref, rel=1e-12)
        assert np.allclose(gpu, ref_pay, rtol=1e-12, atol=1e-12)
    else:
        assert abs(r["price"] - ref) <= 0.1 * se, (r["price"], ref, se)
        S = prob.paths(ids)
        band = tie_band(prob, S, 3e-5)
        check_band(f"parity/{name}", band)
        scale = np.maximum(np.abs(ref_pay), np.max(S, axis=(1, 2)))
        bad = (np.abs(gpu - ref_pay) > 2e-5 * scale) & ~band
        assert not bad.any(), (np.nonzero(bad)[0][:10], gpu[bad][:5], ref_pay[bad][:5])
    assert r["std_err"] == pytest.approx(se, rel=1e-3)
    assert r["n_slots"] == len(prob.days)


def test_c1_full_fp64_matches_oracle_and_black_scholes():
    import paper_2108_03076_amd as P
    from oracle import closed_form as cf
    from oracle.mc import estimate
    cfg = W.C1
    print("[parity] C1 full", flush=True)
    pay = gpu_payoff(cfg)
    r = P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, cfg.n_paths))
    ref, se = estimate(oracle_problem(cfg).payoffs(np.arange(cfg.n_paths)))
    assert r["price"] == pytest.approx(ref, rel=1e-12)
    bs = cf.bs_call(100, 100, 0.03, 0.2, 1.0)
    assert abs(r["price"] - bs) < 3 * r["std_err"]


def test_c3_full_size_sampled_paths():
    """2^20 paths x 1260 days in the launch configuration the benchmark times;
    sampled per-path payoffs against the oracle computed one by one."""
    import paper_2108_03076_amd as P
    from oracle import closed_form as cf
    cfg = W.C3
    n = cfg.n_paths
    print("[parity] C3 full size", flush=True)
    pay = gpu_payoff(cfg)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    for mode, engine in (("fused", "compiled"), ("two_phase", "compiled"), ("fused", "interpreter")):
        r = P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg),
                    **opts_kw(cfg, n, mode=mode, payoffs=out, engine=engine))
        gpu = out.double().cpu().numpy()
        ids = sample_ids(n, 48)
        prob = oracle_problem(cfg)
        ref = prob.payoffs(ids)
        S = prob.paths(ids)
        band = tie_band(prob, S, 3e-5)
        check_band("c3_full", band)
        scale = np.maximum(np.abs(ref), np.max(S, axis=(1, 2)))
        bad = (np.abs(gpu[ids] - ref) > 2e-5 * scale) & ~band
        assert not bad.any(), (mode, ids[bad])
        assert r["sum"] == pytest.approx(gpu.sum(), rel=1e-9)
        bgk = cf.down_and_out_call(100, 100, cf.bgk_barrier(70, 0.3, 1 / 252), 0.03, 0.3, 5.0)
        assert abs(r["price"] - bgk) < 3 * r["std_err"] + 0.02, (r["price"], bgk, r["std_err"])
        assert r["path_dates"] == n * 1260


FULL_SIZE = {"c3": W.C3, "c1": _small(W.C1, n_paths=1 << 20),
             # a ragged count: the fused kernel streams two paths per lane
             # from 2^17 paths, and its last lane holds one real path
             "c3_odd": _small(W.C3, n_paths=(1 << 17) + 3),
             # three correlated assets: the fused kernel's blocks make the step
             # coefficients from their own factorisation, the path generator
             # from the prepared factor; the paths must still agree bit for bit
             "c2": W.C2, "c2_f64": _small(W.C2, precision="f64")}


@pytest.mark.parametrize("name", list(FULL_SIZE))
def test_stored_path_evaluator_at_full_size_equals_fused(name):
    """At 2^20 paths the stored-path evaluator gives each lane 16 FP32 (or
    8 FP64) consecutive paths, and the fused kernel streams two paths per
    lane where the payoff reads forward; every per-path payoff equals the
    fused kernel's bit for bit (the same path values and the same
    operations), also at a ragged path count."""
    import paper_2108_03076_amd as P
    cfg = FULL_SIZE[name]
    n = cfg.n_paths
    print(f"[parity] {name} full size: two-phase against fused", flush=True)
    pay = gpu_payoff(cfg)
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    outs = {}
    for mode in ("fused", "two_phase"):
        out = torch.empty(n, dtype=dt, device="cuda")
        r = P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n, mode=mode, payoffs=out))
        assert r["mode_used"] == (2 if mode == "fused" else 1)
        outs[mode] = (out, r)
    assert torch.equal(outs["fused"][0], outs["two_phase"][0])
    assert outs["fused"][1]["sum"] == pytest.approx(outs["two_phase"][1]["sum"], rel=1e-12)


def test_c2_full_size_sampled_paths():
    import paper_2108_03076_amd as P
    cfg = W.C2
    n = cfg.n_paths
    print("[parity] C2 full size", flush=True)
    pay = gpu_payoff(cfg)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    r = P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n, payoffs=out))
    gpu = out.double().cpu().numpy()
    ids = sample_ids(n, 200)
    prob = oracle_problem(cfg)
    ref = prob.payoffs(ids)
    S = prob.paths(ids)
    band = tie_band(prob, S, 3e-5)
    check_band("c2_full", band)
    bad = (np.abs(gpu[ids] - ref) > 2e-5 * np.maximum(np.abs(ref), 100.0)) & ~band
    assert not bad.any(), ids[bad]
    assert r["sum"] == pytest.approx(gpu.sum(), rel=1e-9)
    # the full-size price against the oracle's on the same 2^20 Sobol points
    # (stored by tests/golden/make_oracle_values.py)
    g = golden()["c2_full_price"]
    assert g["paths"] == n
    print(f"[parity] C2 full price gpu {r['price']:.6f} oracle {g['price']:.6f} se {g['se']:.5f}", flush=True)
    assert abs(r["price"] - g["price"]) <= 0.1 * g["se"], (r["price"], g)


@pytest.mark.parametrize("engine", ["interpreter", "compiled"])
def test_batch_matches_single_and_oracle(engine):
    import paper_2108_03076_amd as P
    from oracle.mc import estimate
    cfg = _small(W.C4)
    T = np.array([20, 45, 7, 33, 60, 1, 0, 52], dtype=np.int32)
    K = np.linspace(90, 110, T.size)
    B = np.linspace(60, 95, T.size)
    n = 1500
    print(f"[parity] batch {engine}", flush=True)
    pay = gpu_payoff(cfg)
    res = P.price_batch(pay, T.reshape(-1, 1), np.stack([K, B], 1), **model_kw(cfg),
                        **opts_kw(cfg, n, engine=engine))
    for i in range(T.size):
        one = P.price(pay, [int(T[i])], [K[i], B[i]], **model_kw(cfg),
                      **opts_kw(cfg, n, instance=i, engine=engine))
        assert res[i]["price"] == pytest.approx(one["price"], rel=1e-12, abs=1e-12)
        prob = oracle_problem(cfg, tenv={"T": int(T[i])}, params=[K[i], B[i]], instance=i)
        ref, se = estimate(prob.payoffs(np.arange(n)))
        assert abs(res[i]["price"] - ref) <= 0.1 * se + 1e-9, (i, res[i]["price"], ref, se)
        assert res[i]["n_slots"] == T[i]


def test_three_asset_batch_matches_single_fused():
    """A batch of worst-of autocalls sharing one template environment runs the
    whole-path kernel with step coefficients made per tile from the prepared
    factors; a single fused price makes them in each block from its own
    factorisation.  The paths are the same, so the prices agree up to the
    order of summation."""
    import paper_2108_03076_amd as P
    cfg = W.C2
    m, n = 4, 4096
    rng = np.random.default_rng(3)
    spot = 100.0 * (1.0 + 0.1 * rng.standard_normal((m, 3)))
    vol = rng.uniform(0.1, 0.4, (m, 3))
    corr = np.stack([np.array(W.corr_equi(3, r)) for r in rng.uniform(0.0, 0.8, m)])
    tenv = np.full((m, 1), cfg.tenv[0], np.int32)
    print("[parity] three-asset batch against single fused", flush=True)
    pay = gpu_payoff(cfg)
    res = P.price_batch(pay, tenv, np.zeros((m, 0)), spot=spot, vol=vol, corr=corr, rate=cfg.rate,
                        years_per_day=cfg.years_per_day, per_instance_model=True, **opts_kw(cfg, n))
    for i in range(m):
        one = P.price(pay, cfg.tenv, [], spot=spot[i], vol=vol[i], corr=corr[i], rate=cfg.rate,
                      years_per_day=cfg.years_per_day, **opts_kw(cfg, n, instance=i, mode="fused"))
        assert one["mode_used"] == 2
        assert res[i]["price"] == pytest.approx(one["price"], rel=1e-12, abs=1e-12), (i, res[i], one)


def test_batch_per_instance_model_and_determinism():
    import paper_2108_03076_amd as P
    from oracle.mc import estimate
    cfg = W.C5
    pts = W.c5_points(6, seed=7)
    n = 2000
    print("[parity] batch per-instance model", flush=True)
    pay = gpu_payoff(cfg)
    tenv = (pts[:, 7].astype(np.int32) - 1).reshape(-1, 1)
    corr = np.stack([np.array(W.corr_equi(3, r)) for r in pts[:, 6]])
    kw = dict(spot=pts[:, 0:3], vol=pts[:, 3:6], corr=corr, rate=cfg.rate, years_per_day=cfg.years_per_day,
              per_instance_model=True)
    a = P.price_batch(pay, tenv, np.zeros((6, 0)), **kw, **opts_kw(cfg, n))
    b = P.price_batch(pay, tenv, np.zeros((6, 0)), **kw, **opts_kw(cfg, n))
    for i in range(6):
        assert a[i]["sum"] == b[i]["sum"] and a[i]["sum_sq"] == b[i]["sum_sq"]
        prob = oracle_problem(cfg, tenv={"N": int(tenv[i, 0])}, spot=pts[i, 0:3], vol=pts[i, 3:6],
                              corr=corr[i], instance=i)
        ref, se = estimate(prob.payoffs(np.arange(n)))
        assert abs(a[i]["price"] - ref) <= 0.1 * se + 1e-9, (i, a[i]["price"], ref, se)


def test_compiled_and_interpreted_payoffs_are_identical():
    """Both engines read the same path values and apply the same binary32
    operations, so per-path payoffs agree bit for bit."""
    import paper_2108_03076_amd as P
    for cfg in (_small(W.C3, tenv=[100]), W.C2, W.C1):
        n = 3000
        pay = gpu_payoff(cfg)
        dt = torch.float64 if cfg.precision == "f64" else torch.float32
        outs = []
        for engine in ("interpreter", "compiled"):
            out = torch.empty(n, dtype=dt, device="cuda")
            P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n, payoffs=out, engine=engine))
            outs.append(out.cpu().numpy())
        assert np.array_equal(outs[0], outs[1]), cfg.name


def test_gpu_cholesky_matches_oracle():
    from gpu_common import ctx
    from oracle.model import cholesky
    g = np.random.default_rng(3)
    mats = []
    for _ in range(5):
        a = g.normal(size=(3, 3))
        mats.append(a @ a.T + 3 * np.eye(3))
    mats = np.stack(mats)
    L = ctx().cholesky(mats)
    for i in range(5):
        assert np.allclose(L[i], cholesky(mats[i]), rtol=1e-14, atol=1e-14)


def test_gpu_error_paths():
    import paper_2108_03076_amd as P
    cfg = W.C2
    pay = gpu_payoff(cfg)
    with pytest.raises(P.PmcError) as e:
        P.price(pay, cfg.tenv, [], **model_kw(cfg, corr=W.corr_equi(3, -0.7)), **opts_kw(cfg, 256))
    assert e.value.name == "E_NOT_PD"
    with pytest.raises(P.PmcError) as e:
        P.price(pay, [-1], [], **model_kw(cfg), **opts_kw(cfg, 256))
    assert e.value.name == "E_TENV"
    with pytest.raises(P.PmcError) as e:
        P.price(pay, [70000], [], **model_kw(cfg), **opts_kw(cfg, 256))
    assert e.value.name == "E_HORIZON"
    with pytest.raises(P.PmcError) as e:
        P.price(pay, cfg.tenv, [], **model_kw(cfg, spot=[100, float("nan"), 100]), **opts_kw(cfg, 256))
    assert e.value.name == "E_ARG"
    # the context still works after errors
    r = P.price(pay, cfg.tenv, [], **model_kw(cfg), **opts_kw(cfg, 256))
    assert math.isfinite(r["price"])


def test_edge_cases_single_path_and_no_slots():
    import paper_2108_03076_amd as P
    from oracle.mc import estimate
    cfg = W.C1
    pay = gpu_payoff(cfg)
    r = P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, 1))
    ref, _ = estimate(oracle_problem(cfg).payoffs(np.arange(1)))
    assert r["price"] == pytest.approx(ref, rel=1e-12)
    # maturity 0: only the spot is read (no simulated day); the call pays max(S0-K,0)
    r = P.price(pay, [0], [90.0], **model_kw(cfg), **opts_kw(cfg, 300))
    assert r["n_slots"] == 0 and r["price"] == pytest.approx(10.0, rel=1e-12)
    # deterministic expression: cash at day 10
    cash = P.Payoff(pay.ctx, "(mult (real 2.0) (payoff 10 X Y))", ["S"])
    r = P.price(cash, [], [], **model_kw(cfg), **opts_kw(cfg, 777))
    assert r["price"] == pytest.approx(2 * math.exp(-0.03 * 10 / 252), rel=1e-12)
    r = P.price(cash, [], [], **model_kw(cfg), **opts_kw(cfg, 777, parties=("Y", "X")))
    assert r["price"] == pytest.approx(-2 * math.exp(-0.03 * 10 / 252), rel=1e-12)
    # the same with Sobol words (no dimension is drawn) in both precisions
    for prec in ("f64", "f32"):
        r = P.price(cash, [], [], **model_kw(cfg), **opts_kw(cfg, 777, rng="sobol", precision=prec))
        assert r["price"] == pytest.approx(2 * math.exp(-0.03 * 10 / 252), rel=1e-6)


@pytest.mark.parametrize("engine", ["interpreter", "compiled"])
def test_time_parameterised_pricing_matches_oracle(engine):
    """cutPayoff (Sec. 4.1) priced at several current times on the GPU against
    the oracle's cut expression on the same stream."""
    import paper_2108_03076_amd as P
    from oracle.il import cut_payoff, parse
    from oracle.mc import estimate
    for cfg, nows in ((_small(W.C3, tenv=[60]), (0, 1, 30, 60, 61)), (W.C2, (0, 1, 3, 5, 6)), (W.C1, (0, 252, 253))):
        n = 2000
        pay = gpu_payoff(cfg).cut()
        for now in nows:
            print(f"[parity] cut {cfg.name} now={now} {engine}", flush=True)
            r = P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n, t_now=now, engine=engine))
            prob = oracle_problem(cfg, il=cut_payoff(parse(cfg.il)), t_now=now)
            ref, se = estimate(prob.payoffs(np.arange(n)))
            if cfg.precision == "f64":
                assert r["price"] == pytest.approx(ref, rel=1e-12, abs=1e-12)
            else:
                assert abs(r["price"] - ref) <= 0.1 * se + 1e-6, (cfg.name, now, r["price"], ref, se)
