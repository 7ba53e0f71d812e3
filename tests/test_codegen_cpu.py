"""The generated payoff source compiles for gfx950 (CPU only: hipcc
cross-compiles; nothing runs)."""
import os
import shutil
import subprocess

import pytest

import workloads as W

hipcc = shutil.which("hipcc")


@pytest.mark.skipif(hipcc is None, reason="hipcc not available")
@pytest.mark.parametrize("name,defs", [("C3", ("float", 0, 1, 1, 1)), ("C2", ("float", 1, 3, 0, 1)),
                                       ("C1", ("double", 0, 1, 0, 1)), ("C3", ("float", 0, 1, 1, 4)),
                                       ("C2", ("float", 1, 3, 1, 4)), ("C1", ("double", 0, 1, 1, 2))])
def test_generated_payoff_compiles(tmp_path, name, defs):
    import paper_2108_03076_amd as P
    cfg = W.CONFIGS[name]
    pay = P.load_payoff(cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)
    src = pay.source()
    assert "struct GenPayoff" in src and "pmc_jit_mc" in src
    f = tmp_path / "payoff.hip"
    f.write_text(src)
    real, rng, a, mem, lanes = defs
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-include", "hip/hip_runtime.h", "-c", str(f),
           "-o", str(tmp_path / "payoff.o"), f"-DPMC_REAL={real}", f"-DPMC_RNG={rng}", f"-DPMC_A={a}",
           f"-DPMC_MEM={mem}", f"-DPMC_P={lanes}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
