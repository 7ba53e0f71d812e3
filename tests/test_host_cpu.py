"""Host side of the library without a GPU: the C ABI's exports, the loader's
error paths and limits, grids, cutPayoff and generated source."""
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pmc_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    import ctypes
    import paper_2108_03076_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(P.EXPORTED) | {"pmc_version"}


def _err(il, assets=("S",), params=(), tvars=()):
    import paper_2108_03076_amd as P
    with pytest.raises(P.PmcError) as e:
        P.load_payoff(il, list(assets), list(params), list(tvars))
    return e.value.name


def test_loader_error_codes():
    assert _err("(add (real 1.0)") == "E_PARSE"
    assert _err("(foo (real 1.0))") == "E_PARSE"
    assert _err("(real 1.0) (real 2.0)") == "E_PARSE"
    assert _err("(add (real 1.0) (nat 1))") == "E_TYPE"
    assert _err("(lt (real 1.0) (real 2.0))") == "E_TYPE"          # not real-valued
    assert _err("(model Q 0)") == "E_TYPE"                         # unknown observable
    assert _err("(payoff (tvar T) X Y)") == "E_TENV"               # undeclared template variable
    assert _err("(real 1.0)", assets=("S", "K"), params=("K",)) == "E_ARG"
    assert _err("(real 1.0)", assets=("A", "B", "C", "D", "E")) == "E_UNSUPPORTED"
    deep = "(real 1.0)"
    for _ in range(9):
        deep = f"(loopif (bool false) (real 1.0) {deep} 1)"
    assert _err(deep) == "E_UNSUPPORTED"                           # loopif nesting > 8


def test_register_limit():
    # a right-deep chain needs one register per level under Sethi-Ullman too
    e = "(real 1.0)"
    for i in range(40):
        e = f"(add (mult (model S {i}) (model S {i + 1})) {e})"
    import paper_2108_03076_amd as P
    p = P.load_payoff(e, ["S"])
    assert p.info()["n_regs"] <= 4                                  # SU evaluates the deep side first
    wide = "(real 1.0)"
    for i in range(34):
        wide = f"(add {wide} (mult (real 2.0) (model S {i})))"
    P.load_payoff(wide, ["S"])


def test_grid_and_limits():
    import paper_2108_03076_amd as P
    p = P.load_payoff(W.DOWN_AND_OUT_CALL, ["S"], ["K", "B"], ["T"])
    days, hz = p.grid([100])
    assert days == list(range(1, 101)) and hz == 100
    with pytest.raises(P.PmcError) as e:
        p.grid([-1])
    assert e.value.name == "E_TENV"
    with pytest.raises(P.PmcError) as e:
        p.grid([70000])
    assert e.value.name == "E_HORIZON"
    q = P.load_payoff(W.WORST_OF_AUTOCALL, ["S1", "S2", "S3"], [], ["N"])
    assert q.grid([4]) == ([1, 2, 3, 4, 5], 5)
    assert q.grid([0]) == ([1], 1)


def test_cut_and_generated_source():
    import paper_2108_03076_amd as P
    p = P.load_payoff(W.EUROPEAN_CALL, ["S"], ["K"], ["T"])
    c = p.cut()
    assert c.info()["n_instr"] > p.info()["n_instr"]
    assert c.grid([252]) == p.grid([252])
    src = c.source()
    assert "D.t_now" in src and "pmc_jit_mc" in src
    assert "D.t_now" not in p.source().split("struct GenPayoff")[1]


def test_streamed_reads():
    """Which expressions read their dates in non-decreasing order (their
    paths can be generated as a stream): the down-and-out and the European
    call do, at any maturity and after a history; the worst-of autocall's
    maturity branch looks back three dates and does not, nor does a loop
    that reads the day before its shift after its shift (one that reads it
    first does: the shift's day is then the newest slot)."""
    import paper_2108_03076_amd as P
    for cfg, envs in ((W.C3, ([1260], [60], [0])), (W.C1, ([252],)), (W.C4, ([252], [1000]))):
        pay = P.load_payoff(cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)
        for env in envs:
            assert pay.streams(env), (cfg.name, env)
            assert pay.streams(env, sim_from=5), (cfg.name, env)
    c2 = W.C2
    pay = P.load_payoff(c2.il, c2.asset_labels, c2.param_labels, c2.tvars)
    assert not pay.streams(c2.tenv)
    fwd = P.load_payoff("(loopif (lt (model S (int -1)) (model S 0)) (payoff 0 X Y) (real 0.0) 30)", ["S"])
    assert fwd.streams([])
    back = P.load_payoff("(loopif (lt (model S 0) (model S (int -1))) (payoff 0 X Y) (real 0.0) 30)", ["S"])
    assert not back.streams([])
    # the same read after a history that covers it: no simulated slot is revisited
    assert back.streams([], sim_from=40)
