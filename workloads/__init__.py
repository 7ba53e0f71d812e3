"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *describes* workloads: payoff-expression text, model
parameters, path counts and seeded parameter draws.  It holds none of the
method's arithmetic (no random streams, no paths, no payoff evaluation), so
the GPU library and the CPU oracle can both take their inputs from here
without sharing code.

The paper's own benchmark contracts (a vanilla call, a discrete barrier
option on three underlyings and a double option; Table 1, Sec. 6.2) and the
engine's market data are not published with it.  The configurations below
stand in for them with the same shapes:

* C1  European call on 1 asset, 1 observation day, FP64 (vanilla stand-in).
* C2  worst-of autocall on 3 correlated assets, 5 annual dates, loopif
      early redemption and a knock-in (discrete barrier stand-in).
* C3  down-and-out call on 1 asset monitored daily for 1260 days.
* C4  1024 templated instances of the C3 contract (maturity, strike and
      barrier drawn per instance).
* C5  the C2 family with per-point model parameters, for the surrogate.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Payoff expressions (the IL text syntax documented in include/pmc.h)
# ---------------------------------------------------------------------------

# Example 1 of the paper with strike and maturity abstracted (Sec. 2): pay
# (S_T - K) at day T when S_T > K.  K is a parameter observable.
EUROPEAN_CALL = """
(if (lt (model K 0) (model S (tvar T)))
    (mult (sub (model S (tvar T)) (model K 0)) (payoff (tvar T) X Y))
    (real 0.0))
"""

# Daily-monitored down-and-out call: loopif checks S <= B on days 0..T; if it
# never knocks out, the call pays at day T (the loopif shift is then T).
DOWN_AND_OUT_CALL = """
(loopif (leq (model S 0) (model B 0))
        (real 0.0)
        (if (lt (model K 0) (model S 0))
            (mult (sub (model S 0) (model K 0)) (payoff 0 X Y))
            (real 0.0))
        (tvar T))
"""


# Forward contract: pays S_T - K at day T (linear in the spot on every path).
FORWARD = """
(mult (sub (model S (tvar T)) (model K 0)) (payoff (tvar T) X Y))
"""

# Two-asset basket call: pays (S1_T + S2_T)/2 - K at day T when positive.
BASKET_CALL = """
(if (lt (model K 0) (mult (real 0.5) (add (model S1 (tvar T)) (model S2 (tvar T)))))
    (mult (sub (mult (real 0.5) (add (model S1 (tvar T)) (model S2 (tvar T)))) (model K 0))
          (payoff (tvar T) X Y))
    (real 0.0))
"""


# Double option (the paper's third benchmark contract, Table 1): two
# European calls on a two-asset model, both paying at day T.
DOUBLE_CALL = """
(add (if (lt (model K1 0) (model S1 (tvar T)))
         (mult (sub (model S1 (tvar T)) (model K1 0)) (payoff (tvar T) X Y))
         (real 0.0))
     (if (lt (model K2 0) (model S2 (tvar T)))
         (mult (sub (model S2 (tvar T)) (model K2 0)) (payoff (tvar T) X Y))
         (real 0.0)))
"""


def _worst(day):
    """min over the three assets on a day offset (an ILTExprZ)."""
    return f"(min (min (model S1 {day}) (model S2 {day})) (model S3 {day}))"


# Worst-of autocall on 3 assets, annual observation dates 1 .. N+1 (N is the
# template variable).  W(k) = min_a S_a(k) / 100 with reference level 100 and
# notional 100.  On the first date with W >= 1 it redeems, paying 105 on that
# date.  Otherwise at maturity it pays 100 W(N+1) if W < 0.6 was seen on any
# of the observation dates (knock-in), else 100.  The maturity branch runs
# with loop shift N and looks back with offsets 1, 0, -1, -2, -3: days N+1 ..
# N-3.  Offsets that reach day 0 or earlier read the spot, which never knocks
# in while every spot is >= 60.
def _or_chain(terms):
    """Right-nested (or t1 (or t2 (... tn)))."""
    return terms[0] if len(terms) == 1 else f"(or {terms[0]} {_or_chain(terms[1:])})"


_KNOCK_IN = _or_chain([f"(lt {_worst(o)} (real 60.0))"
                       for o in ("1", "0", "(int -1)", "(int -2)", "(int -3)")])

WORST_OF_AUTOCALL = f"""
(loopif (leq (real 100.0) {_worst("1")})
        (mult (real 105.0) (payoff 1 X Y))
        (if {_KNOCK_IN}
            (mult {_worst("1")} (payoff 1 X Y))
            (mult (real 100.0) (payoff 1 X Y)))
        (tvar N))
"""


@dataclass
class Config:
    name: str
    il: str
    asset_labels: list
    param_labels: list
    params: list
    tvars: list
    tenv: list
    spot: list
    vol: list
    corr: list | None
    rate: float
    years_per_day: float
    n_paths: int
    rng: str = "philox"
    seed: int = 42
    precision: str = "f32"
    parties: tuple = ("X", "Y")
    notes: dict = field(default_factory=dict)

    def tenv_dict(self):
        return dict(zip(self.tvars, self.tenv))


def corr_equi(n, rho):
    c = np.full((n, n), float(rho))
    np.fill_diagonal(c, 1.0)
    return c.tolist()


C1 = Config(
    name="C1 european call, 1 asset, 1 date, fp64",
    il=EUROPEAN_CALL, asset_labels=["S"], param_labels=["K"], params=[100.0],
    tvars=["T"], tenv=[252], spot=[100.0], vol=[0.2], corr=None, rate=0.03,
    years_per_day=1.0 / 252.0, n_paths=1 << 16, rng="philox", seed=42, precision="f64")

C2 = Config(
    name="C2 worst-of autocall, 3 assets, 5 annual dates, sobol",
    il=WORST_OF_AUTOCALL, asset_labels=["S1", "S2", "S3"], param_labels=[], params=[],
    tvars=["N"], tenv=[4], spot=[100.0, 100.0, 100.0], vol=[0.15, 0.20, 0.25],
    corr=corr_equi(3, 0.5), rate=0.03, years_per_day=1.0, n_paths=1 << 20, rng="sobol",
    precision="f32")

C3 = Config(
    name="C3 down-and-out call, 1260 daily dates",
    il=DOWN_AND_OUT_CALL, asset_labels=["S"], param_labels=["K", "B"], params=[100.0, 70.0],
    tvars=["T"], tenv=[1260], spot=[100.0], vol=[0.3], corr=None, rate=0.03,
    years_per_day=1.0 / 252.0, n_paths=1 << 20, rng="philox", seed=42, precision="f32")


C2D = Config(
    name="double call, 2 assets (rho 0.5), 1 date, philox",
    il=DOUBLE_CALL, asset_labels=["S1", "S2"], param_labels=["K1", "K2"], params=[100.0, 95.0],
    tvars=["T"], tenv=[252], spot=[100.0, 100.0], vol=[0.2, 0.3], corr=corr_equi(2, 0.5), rate=0.03,
    years_per_day=1.0 / 252.0, n_paths=1 << 20, rng="philox", seed=42, precision="f32")


def c4_instances(n_inst=1024, seed=42):
    """Per-instance template values and parameters for the batched workload:
    T days uniform in {252..1260}, K uniform in [80, 120], barrier b*100 with
    b uniform in [0.5, 0.8] (numpy default_rng(seed), drawn in that order)."""
    g = np.random.default_rng(seed)
    T = g.integers(252, 1260, size=n_inst, endpoint=True).astype(np.int32)
    K = g.uniform(80.0, 120.0, size=n_inst)
    b = g.uniform(0.5, 0.8, size=n_inst)
    return T, K, b * 100.0


C4 = Config(
    name="C4 1024 templated down-and-out calls, 252-1260 daily dates",
    il=DOWN_AND_OUT_CALL, asset_labels=["S"], param_labels=["K", "B"], params=[100.0, 70.0],
    tvars=["T"], tenv=[1260], spot=[100.0], vol=[0.2], corr=None, rate=0.03,
    years_per_day=1.0 / 252.0, n_paths=1 << 16, rng="philox", seed=42, precision="f32",
    notes={"n_instances": 1024})

# Surrogate input box (spots, vols, pairwise correlation, number of annual
# observation dates) for the worst-of autocall family.
C5_BOX = {"spot": (70.0, 130.0), "vol": (0.10, 0.40), "rho": (0.0, 0.9), "n_obs": (1, 5)}


def c5_points(n, seed):
    """Surrogate inputs: [n, 8] = (S1, S2, S3, v1, v2, v3, rho, n_obs)."""
    g = np.random.default_rng(seed)
    s = g.uniform(*C5_BOX["spot"], size=(n, 3))
    v = g.uniform(*C5_BOX["vol"], size=(n, 3))
    r = g.uniform(*C5_BOX["rho"], size=(n, 1))
    m = g.integers(C5_BOX["n_obs"][0], C5_BOX["n_obs"][1], size=(n, 1), endpoint=True)
    return np.concatenate([s, v, r, m.astype(np.float64)], axis=1)


C5 = Config(
    name="C5 surrogate over the worst-of autocall family",
    il=WORST_OF_AUTOCALL, asset_labels=["S1", "S2", "S3"], param_labels=[], params=[],
    tvars=["N"], tenv=[4], spot=[100.0, 100.0, 100.0], vol=[0.15, 0.20, 0.25],
    corr=corr_equi(3, 0.5), rate=0.03, years_per_day=1.0, n_paths=1 << 16, rng="philox",
    seed=42, precision="f32", notes={"train_points": 1 << 20, "test_points": 4096,
                                     "judge_paths": 1 << 22, "infer_batch": 65536})

CONFIGS = {"C1": C1, "C2": C2, "C2D": C2D, "C3": C3, "C4": C4, "C5": C5}


# Risk workload: bump-and-revalue Greeks (delta, gamma per spot; vega per
# volatility) of the C4 instruments by central differences on common random
# numbers; spot bumps are relative, volatility bumps absolute.
RISK_BUMPS = {"rel_spot_bump": 0.01, "abs_vol_bump": 0.01}
