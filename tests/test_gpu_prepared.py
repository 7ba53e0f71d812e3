"""Repeated single pricings: a call whose inputs are byte-identical to the
previous one reuses its host-side preparation (tables, launch arguments,
kernel), and every kernel runs again.  These tests check that reuse never
returns a stale answer: the results of an identical repeat are bit-identical
to a fresh call, and any change of an input, of the device tables (another
payoff or a batch in between) or of the payoff object itself is seen."""
import numpy as np
import pytest

import workloads as W
from gpu_common import ctx, gpu_payoff, model_kw, opts_kw

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fresh(pay, cfg, n, **over):
    import paper_2108_03076_amd as P
    return P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg, **over), **opts_kw(cfg, n))


def test_identical_repeat_is_bit_identical_and_inputs_changed_in_place_are_seen():
    import paper_2108_03076_amd as P
    cfg, n = W.C2, 1 << 16
    pay = gpu_payoff(cfg)
    print("[prepared] repeat and in-place change", flush=True)
    pr = P.Pricer(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n))
    first = pr().as_dict()
    for _ in range(3):
        again = pr().as_dict()
        assert (again["sum"], again["sum_sq"]) == (first["sum"], first["sum_sq"])
    ref = _fresh(pay, cfg, n)
    assert (ref["sum"], ref["sum_sq"]) == (first["sum"], first["sum_sq"])
    # the Pricer's own spot array, changed in place: same pointer, new value
    pr._keep[0][0] = 90.0
    moved = pr().as_dict()
    ref2 = _fresh(pay, cfg, n, spot=[90.0] + list(cfg.spot[1:]))
    assert (moved["sum"], moved["sum_sq"]) == (ref2["sum"], ref2["sum_sq"])
    assert moved["price"] != first["price"]


def test_tables_rewritten_between_identical_calls():
    """Another payoff's pricing and a batch upload their own tables between
    two identical calls; the second call must rebuild, not reuse."""
    import paper_2108_03076_amd as P
    cfg, n = W.C2, 1 << 16
    pay = gpu_payoff(cfg)
    print("[prepared] interleaved tables", flush=True)
    pr = P.Pricer(pay, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, n))
    first = pr().as_dict()
    c1 = W.C1
    other = gpu_payoff(c1)
    _fresh(other, c1, 4096)
    again = pr().as_dict()
    assert (again["sum"], again["sum_sq"]) == (first["sum"], first["sum_sq"])
    c4 = W.C4
    pay4 = gpu_payoff(c4)
    T = np.array([[20], [40], [60]], dtype=np.int32)
    P.price_batch(pay4, T, np.tile(np.array(c4.params), (3, 1)), **model_kw(c4), **opts_kw(c4, 2048))
    again = pr().as_dict()
    assert (again["sum"], again["sum_sq"]) == (first["sum"], first["sum_sq"])


def test_new_payoff_object_is_never_mistaken_for_a_freed_one():
    """A payoff freed and a new one loaded (possibly at the same address):
    the new object's call compiles and runs its own kernel."""
    import gc
    import paper_2108_03076_amd as P
    cfg, n = W.C2, 1 << 14
    print("[prepared] payoff replaced", flush=True)
    pay = gpu_payoff(cfg)
    a = _fresh(pay, cfg, n)
    del pay
    gc.collect()
    c1 = W.C1
    pay1 = P.Payoff(ctx(), c1.il, c1.asset_labels, c1.param_labels, c1.tvars)
    b = P.price(pay1, c1.tenv, c1.params, **model_kw(c1), **opts_kw(c1, n))
    ref = _fresh(pay1, c1, n)
    assert (b["sum"], b["sum_sq"]) == (ref["sum"], ref["sum_sq"])
    assert b["price"] != a["price"]


def test_repeated_batch_reuses_its_plan_and_sees_every_change():
    """A batch call whose inputs equal the previous one's replays its plan:
    sums bit-identical to the first call; an input changed in place (same
    arrays), another payoff's pricing in between, or another tile (forced
    block) is seen and priced afresh."""
    import paper_2108_03076_amd as P
    cfg = W.C4
    pay = gpu_payoff(cfg)
    T = np.array([[30], [60], [45], [90]], dtype=np.int32)
    KB = np.array([[95.0, 70.0], [100.0, 72.0], [105.0, 68.0], [110.0, 75.0]])
    kw = dict(**model_kw(cfg), **opts_kw(cfg, 4096))
    print("[prepared] batch repeat", flush=True)
    first = P.price_batch(pay, T, KB, **kw)
    for _ in range(3):
        again = P.price_batch(pay, T, KB, **kw)
        assert [(r["sum"], r["sum_sq"]) for r in again] == [(r["sum"], r["sum_sq"]) for r in first]
    KB[2, 1] = 90.0          # in place: the same array, a new barrier
    moved = P.price_batch(pay, T, KB, **kw)
    fresh = P.price_batch(pay, T.copy(), KB.copy(), **dict(kw, block=128))
    assert moved[2]["sum"] != first[2]["sum"]
    for a, b in zip(moved, fresh):
        assert a["sum"] == pytest.approx(b["sum"], rel=1e-12, abs=1e-9)
    assert [r["sum"] for i, r in enumerate(moved) if i != 2] == [r["sum"] for i, r in enumerate(first) if i != 2]
    c1 = W.C1
    _fresh(gpu_payoff(c1), c1, 4096)
    again = P.price_batch(pay, T, KB, **kw)
    assert [r["sum"] for r in again] == [r["sum"] for r in moved]
