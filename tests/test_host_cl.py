"""The library's contract-language front end (pmc_contract_compile /
pmc_contract_load, C++) on the CPU: Example 3 compiles to the expression
the paper prints; on random contracts it agrees with the oracle's own
compiler (written separately, in Python) by value on random scenarios and
by simulated grid; the workload contracts written in CL give the workloads'
payoff expressions; malformed contracts are refused."""
import math

import numpy as np
import pytest

import workloads as W
from golden_io import all_fixtures, load
from oracle import cl, grid
from oracle.il import il_eval, parse
from test_oracle_cl import rand_contract, rand_env


def to_cl(c):
    """A contract tuple of the oracle as contract-language text (operators
    in prefix form, literals as numbers)."""
    def t(x):
        return str(x[1]) if x[0] == "n" else x[1]

    def e(x):
        if x[0] == "obs":
            return f"obs({x[1]}, {x[2]})"
        if x[0] == "lit":
            return repr(float(x[1]))
        if x[0] == "blit":
            return "true" if x[1] else "false"
        return f"{x[1]}({', '.join(e(a) for a in x[2:])})"

    k = c[0]
    if k == "zero":
        return "zero"
    if k == "transfer":
        return f"transfer({c[1]}, {c[2]})"
    if k == "scale":
        return f"scale({e(c[1])}, {to_cl(c[2])})"
    if k == "translate":
        return f"translate({t(c[1])}, {to_cl(c[2])})"
    if k == "both":
        return f"both({to_cl(c[1])}, {to_cl(c[2])})"
    return f"ifWithin({e(c[1])}, {t(c[2])}, {to_cl(c[3])}, {to_cl(c[4])})"


def _same_values(il_a, il_b, tenvs, params=None, seeds=range(6), labels=("S",), parties=("X", "Y")):
    for seed in seeds:
        g = np.random.default_rng(seed)
        tab = {(l, d): float(g.lognormal(np.log(100), 0.25)) for l in labels for d in range(-12, 140)}
        rho = lambda l, d: (params or {}).get(l) if l in (params or {}) else tab[(l, d)]
        disc = lambda k: 0.999 ** k
        for delta in tenvs:
            for now in (0, 3):
                a = il_eval(il_a, rho, delta, 0, now, disc, *parties)
                b = il_eval(il_b, rho, delta, 0, now, disc, *parties)
                assert a == pytest.approx(b, rel=1e-13, abs=1e-13), (delta, now, a, b)


def test_example3_compiles_to_the_printed_expression():
    import paper_2108_03076_amd as P
    text = """
      translate(t0,
        both(scale(100.0, transfer(you, me)),
             translate(t1,
               if(obs(AAPL, 0) > 100.0,
                  scale(obs(AAPL, 0) - 100.0, transfer(you, me, USD)),
                  zero))))
    """
    rec = load(all_fixtures("example3")[0])
    assert parse(P.compile_contract(text)) == parse(rec["il"])


@pytest.mark.parametrize("seed", range(30))
def test_random_contracts_agree_with_the_oracle_compiler(seed):
    import paper_2108_03076_amd as P
    g = np.random.default_rng(9000 + seed)
    c = rand_contract(g, 4)
    lib_il = parse(P.compile_contract(to_cl(c)))
    ref_il = cl.compile_contract(c)
    tenvs = [{"a": int(g.integers(0, 6)), "b": int(g.integers(0, 6))} for _ in range(3)]
    _same_values(lib_il, ref_il, tenvs)
    for delta in tenvs:
        assert grid.slots(lib_il, delta, ["S"]) == grid.slots(ref_il, delta, ["S"])
        assert grid.horizon(lib_il, delta) == grid.horizon(ref_il, delta)
    pay = P.load_contract(to_cl(c), ["S"], [], ["a", "b"])
    assert pay.grid([tenvs[0]["a"], tenvs[0]["b"]])[0] == grid.slots(ref_il, tenvs[0], ["S"])


WORST = "min(min(obs(S1, {k}), obs(S2, {k})), obs(S3, {k}))"
PAY1 = "translate(1, transfer(X, Y))"
CONTRACTS = {
    "european": ("translate(T, if(obs(S, 0) > obs(K, 0), scale(obs(S, 0) - obs(K, 0), transfer(X, Y)), zero))",
                 W.C1),
    "down_and_out": ("ifWithin(obs(S, 0) <= obs(B, 0), T, zero,\n"
                     "         if(obs(S, 0) > obs(K, 0), scale(obs(S, 0) - obs(K, 0), transfer(X, Y)), zero))",
                     W.C3),
    "double": ("translate(T, all[if(obs(S1, 0) > obs(K1, 0), scale(obs(S1, 0) - obs(K1, 0), transfer(X, Y)), zero),\n"
               "                 if(obs(S2, 0) > obs(K2, 0), scale(obs(S2, 0) - obs(K2, 0), transfer(X, Y)), zero)])",
               W.C2D),
    "worst_of_autocall": (
        f"ifWithin(100.0 <= {WORST.format(k=1)}, N, scale(105.0, {PAY1}),\n"
        f"  if({' || '.join(WORST.format(k=k) + ' < 60.0' for k in (1, 0, -1, -2, -3))},\n"
        f"     scale({WORST.format(k=1)}, {PAY1}), scale(100.0, {PAY1})))", W.C2),
}


@pytest.mark.parametrize("name", sorted(CONTRACTS))
def test_workload_contracts_compile_to_the_workload_expressions(name):
    """Each workload's payoff expression is the compiled form of a CL
    contract: equal values on random scenarios and template environments,
    the same simulated grid through the library's loader."""
    import paper_2108_03076_amd as P
    text, cfg = CONTRACTS[name]
    lib_il = parse(P.compile_contract(text))
    hand = parse(cfg.il)
    params = dict(zip(cfg.param_labels, cfg.params))
    tv = cfg.tvars[0]
    tenvs = [{tv: v} for v in (0, 1, 4, 30)]
    _same_values(lib_il, hand, tenvs, params=params, labels=cfg.asset_labels)
    a = P.load_contract(text, cfg.asset_labels, cfg.param_labels, cfg.tvars)
    b = P.load_payoff(cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)
    for v in (0, 4, 30):
        assert a.grid([v]) == b.grid([v])


def test_malformed_contracts_are_refused():
    import paper_2108_03076_amd as P
    for bad in ("", "scale(1.0 transfer(a, b))", "translate(-1, zero)", "translate(1.5, zero)",
                "both(zero)", "ifWithin(true, T, zero)", "scale(obs(S, 0.5), zero)", "frobnicate(zero)",
                "zero zero", "scale(1 = 2, zero)", "all[]", "scale(1.0.0, zero)",
                # numerals beyond 31 bits, nesting beyond the limit (refused, never a crash)
                "translate(99999999999999999999, zero)", "scale(obs(S, 4294967296), zero)",
                "scale(1.0, " * 1001 + "zero" + ")" * 1001, "scale(" + "-" * 5000 + "1.0, zero)"):
        with pytest.raises(P.PmcError) as e:
            P.compile_contract(bad)
        assert e.value.name == "E_PARSE", bad
    # well formed but ill typed for the loader: a boolean scale, an unknown label
    with pytest.raises(P.PmcError) as e:
        P.load_contract("scale(true, transfer(X, Y))", ["S"])
    assert e.value.name == "E_TYPE"
    with pytest.raises(P.PmcError) as e:
        P.load_contract("scale(obs(Q, 0), transfer(X, Y))", ["S"])
    assert e.value.name == "E_TYPE"
