"""Named workload variants shared by the GPU parity tests and the script that
writes their stored oracle values (tests/golden/make_oracle_values.py).
Descriptions only: configurations from `workloads`, no arithmetic."""
import dataclasses

import numpy as np

import workloads as W


def small(cfg, **over):
    return dataclasses.replace(cfg, **over)


# Parity cases priced and evaluated at a few thousand paths.
PARITY = {
    "c3_short": small(W.C3, tenv=[37]),
    "c2": W.C2,
    "c1": W.C1,
    "c2_philox": small(W.C2, rng="philox"),
    "c2d": W.C2D,
    # 12 dates x 3 assets: more prices than the compiled engine holds whole,
    # so it slides its window and regenerates on the knock-in's backward reads
    "c2_long": small(W.C2, tenv=[11]),
    # FP64 paths held whole (15 prices in a 16-entry window of register pairs)
    "c2_f64": small(W.C2, precision="f64"),
}

NESTED = """
(loopif (lt (model S 0) (real 92.0))
        (mult (real 1.0) (payoff 0 X Y))
        (loopif (leq (real 108.0) (model S 0))
                (mult (sub (model S 0) (real 100.0)) (payoff 0 X Y))
                (mult (real 0.5) (payoff 0 X Y))
                (tvar M))
        (tvar N))
"""

OPERATORS = """
(if (and (not (lt (model S 2) (real 95.0))) (leq (now) (t (tvar T))))
    (mult (max (div (model S 2) (model S (int -1))) (neg (real 0.5))) (payoff (tvar T) X Y))
    (if (or (eq (model S 1) (real 100.0)) (lt (model S 1) (real 99.0)))
        (mult (min (model S 1) (real 80.0)) (payoff 1 Y X))
        (real 0.0)))
"""


def _program(il, tvars, tenv, precision="f32"):
    return dataclasses.replace(W.C3, il=il, tvars=tvars, tenv=tenv, param_labels=[], params=[],
                               years_per_day=1.0 / 12.0, precision=precision, name="program")


PROGRAMS = {
    "nested": _program(NESTED, ["N", "M"], [3, 2]),
    "nested_zero_inner": _program(NESTED, ["N", "M"], [4, 0]),
    "nested_f64": _program(NESTED, ["N", "M"], [3, 2], precision="f64"),
    "operators": _program(OPERATORS, ["T"], [4]),
}

# Full-size workloads whose sampled paths the tests compare one by one.
FULL = {"c3_full": W.C3, "c2_full": W.C2}

# FP32 cases whose per-path comparisons exclude the tie-band, by the name
# under which the stored band rate is kept.
BAND_CASES = {**{f"parity/{k}": v for k, v in PARITY.items() if v.precision == "f32"},
              **{f"programs/{k}": v for k, v in PROGRAMS.items() if v.precision == "f32"},
              **FULL}


def c4_sample(n_pick=16):
    """Instances of the 1024-instance batched workload spanning its date
    range: the ones at evenly spaced ranks of T (the shortest and the
    longest included).  Returns (ids, T, K, B) with the instances' original
    indices, which are their Philox counter words."""
    T, K, B = W.c4_instances(1024, 42)
    order = np.argsort(T, kind="stable")
    ranks = np.unique(np.round(np.linspace(0, T.size - 1, n_pick)).astype(int))
    ids = order[ranks]
    return ids.astype(np.int64), T[ids], K[ids], B[ids]


C4_SAMPLE_PATHS = 1 << 12
# Full-size instances (2^16 paths each) compared with the full batch.
C4_FULL_PICK = 6
