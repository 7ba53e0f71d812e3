"""Payoff programs beyond the benchmark contracts, through both engines and
both evaluation modes: a loopif nested in another's second branch, a loopif
of count zero, time values and `now`, division, max, equality, not, neg,
or, and, reversed parties and a read before day 0.  The compiled kernels
here are generated for each template environment (loops written out); their
per-path payoffs must equal the interpreter's bit for bit (the same binary32
or binary64 operations in the same order) and the oracle's within the FP32
bars of the parity tests (FP64: 1e-12 relative)."""
import numpy as np
import pytest

from cases import PROGRAMS
from gpu_common import check_band, ctx, gpu_payoff, model_kw, opts_kw, oracle_problem, tie_band

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = PROGRAMS


@pytest.mark.parametrize("name", list(CASES))
def test_program_engines_modes_and_oracle(name):
    import paper_2108_03076_amd as P
    cfg = CASES[name]
    n = 3000
    print(f"[programs] {name}", flush=True)
    pay = gpu_payoff(cfg)
    src = pay.source(cfg.tenv).split("struct GenPayoff")[1]
    assert "read_obs(" not in src   # generated for the environment, loops written out
    dt = torch.float64 if cfg.precision == "f64" else torch.float32
    outs = {}
    for mode, engine in (("fused", "compiled"), ("fused", "interpreter"), ("two_phase", "compiled")):
        out = torch.empty(n, dtype=dt, device="cuda")
        r = P.price(pay, cfg.tenv, cfg.params, **model_kw(cfg),
                    **opts_kw(cfg, n, mode=mode, engine=engine, payoffs=out))
        outs[(mode, engine)] = (out.double().cpu().numpy(), r)
    base = outs[("fused", "compiled")][0]
    for k, (v, r) in outs.items():
        assert np.array_equal(v, base), k
        assert r["sum"] == pytest.approx(base.sum(), rel=1e-12, abs=1e-9)
    prob = oracle_problem(cfg)
    ids = np.arange(n)
    ref = prob.payoffs(ids)
    if cfg.precision == "f64":
        assert np.allclose(base, ref, rtol=1e-12, atol=1e-12)
    else:
        S = prob.paths(ids)
        band = tie_band(prob, S, 3e-5)
        check_band(f"programs/{name}", band)
        scale = np.maximum(np.abs(ref), np.max(S, axis=(1, 2)))
        bad = (np.abs(base - ref) > 2e-5 * scale) & ~band
        assert not bad.any(), (np.nonzero(bad)[0][:10], base[bad][:5], ref[bad][:5])
    assert np.any(base != 0.0)


def test_contracts_loaded_from_the_contract_language_price_as_their_expressions():
    """A workload contract loaded from contract-language text (compiled by
    the library's front end) prices exactly as the workload's hand-written
    payoff expression on the same stream, in both engines."""
    import dataclasses
    import paper_2108_03076_amd as P
    from test_host_cl import CONTRACTS
    for name in sorted(CONTRACTS):
        text, cfg = CONTRACTS[name]
        if cfg.tvars == ["T"] and cfg.tenv[0] > 300:
            cfg = dataclasses.replace(cfg, tenv=[60])
        a = P.load_contract(text, cfg.asset_labels, cfg.param_labels, cfg.tvars, ctx=ctx())
        b = gpu_payoff(cfg)
        for engine in ("interpreter", "compiled"):
            print(f"[contract] {name} {engine}", flush=True)
            ra = P.price(a, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, 3000, engine=engine))
            rb = P.price(b, cfg.tenv, cfg.params, **model_kw(cfg), **opts_kw(cfg, 3000, engine=engine))
            assert (ra["sum"], ra["sum_sq"]) == (rb["sum"], rb["sum_sq"]), (name, engine, ra, rb)
