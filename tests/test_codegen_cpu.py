"""The generated payoff source compiles for gfx950 (CPU only: hipcc
cross-compiles; nothing runs)."""
import os
import shutil
import subprocess

import pytest

import workloads as W

hipcc = shutil.which("hipcc")


@pytest.mark.skipif(hipcc is None, reason="hipcc not available")
@pytest.mark.parametrize("name,defs", [("C3", ("float", 0, 1, 1, 1, 0)), ("C2", ("float", 1, 3, 0, 1, 0)),
                                       ("C1", ("double", 0, 1, 0, 1, 0)), ("C3", ("float", 0, 1, 1, 4, 0)),
                                       ("C2", ("float", 1, 3, 1, 4, 0)), ("C1", ("double", 0, 1, 1, 2, 0)),
                                       ("C2", ("float", 1, 3, 0, 1, 16)), ("C1", ("double", 0, 1, 0, 1, 1)),
                                       ("C2", ("double", 0, 3, 0, 1, 16)), ("C3", ("float", 0, 1, 1, 16, 0)),
                                       ("C1", ("double", 0, 1, 1, 8, 0)),
                                       # one instrument, each block factoring its own matrix
                                       ("C2", ("float", 1, 3, 0, 1, 16, 1, 1)),
                                       ("C1", ("double", 0, 1, 0, 1, 1, 1, 1)),
                                       ("C3", ("float", 0, 1, 0, 1, 0, 1, 1)),
                                       # one instrument from stored paths (prepared factor)
                                       ("C3", ("float", 0, 1, 1, 16, 0, 1, 0)),
                                       # streamed paths: one or two per lane, batch or one instrument
                                       ("C3", ("float", 0, 1, 0, 1, 0, 0, 0, 1)),
                                       ("C3", ("float", 0, 1, 0, 2, 0, 0, 0, 1)),
                                       ("C1", ("double", 0, 1, 0, 2, 0, 1, 1, 1)),
                                       ("C2D", ("float", 0, 2, 0, 4, 0, 0, 0, 1))])
def test_generated_payoff_compiles(tmp_path, name, defs):
    import paper_2108_03076_amd as P
    cfg = W.CONFIGS[name]
    pay = P.load_payoff(cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)
    src = pay.source()
    assert "struct GenPayoff" in src and "pmc_jit_mc" in src
    f = tmp_path / "payoff.hip"
    f.write_text(src)
    real, rng, a, mem, lanes, full, single, own, stream = (defs + (0, 0, 0))[:9]
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-include", "hip/hip_runtime.h", "-c", str(f),
           "-o", str(tmp_path / "payoff.o"), f"-DPMC_REAL={real}", f"-DPMC_RNG={rng}", f"-DPMC_A={a}",
           f"-DPMC_MEM={mem}", f"-DPMC_P={lanes}", f"-DPMC_FULL={full}", f"-DPMC_SINGLE={single}",
           f"-DPMC_OWN={own}", f"-DPMC_STREAM={stream}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]


@pytest.mark.skipif(hipcc is None, reason="hipcc not available")
def test_whole_path_headline_kernel_fits_eight_waves(tmp_path):
    """The worst-of autocall generated for its template environment, with its
    path held whole (5 dates x 3 assets in a 16-entry window) and priced as
    one instrument (no batch queue, each block factoring its own matrix),
    compiles at eight waves per SIMD without scratch memory, and its code
    (the generation exists once) stays far below the 64 KB instruction
    cache."""
    import re
    import paper_2108_03076_amd as P
    cfg = W.CONFIGS["C2"]
    pay = P.load_payoff(cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)
    f = tmp_path / "payoff.hip"
    f.write_text(pay.source(cfg.tenv))
    out = tmp_path / "payoff.s"
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-include", "hip/hip_runtime.h", "--cuda-device-only", "-S", str(f), "-o", str(out),
           "-DPMC_REAL=float", "-DPMC_RNG=1", "-DPMC_A=3", "-DPMC_MEM=0", "-DPMC_P=1", "-DPMC_FULL=16",
           "-DPMC_WAVES=8", "-DPMC_SINGLE=1", "-DPMC_OWN=1"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    asm = out.read_text()
    assert re.search(r"; ScratchSize: 0\b", asm)
    assert re.search(r"; Occupancy: 8\b", asm)
    code = int(re.search(r"; codeLenInByte = (\d+)", asm).group(1))
    assert code < 32 * 1024, code


def test_source_for_a_template_environment():
    """Generated for a known environment, the autocall's five loopif
    iterations are written out and read fixed slots (no run-time day
    lookups); a loop too long to write out keeps the generic form."""
    import paper_2108_03076_amd as P
    cfg = W.CONFIGS["C2"]
    pay = P.load_payoff(cfg.il, cfg.asset_labels, cfg.param_labels, cfg.tvars)
    gen, spec = pay.source(), pay.source(cfg.tenv)
    body = spec.split("struct GenPayoff")[1]
    assert "read_obs(" not in body and "for (;;)" not in body
    assert body.count("do {") == 1 and body.count("if (vall(done_") == cfg.tenv[0] + 1
    assert "read_obs(" in gen.split("struct GenPayoff")[1]
    c3 = W.CONFIGS["C3"]
    pay3 = P.load_payoff(c3.il, c3.asset_labels, c3.param_labels, c3.tvars)
    assert "read_obs(" in pay3.source(c3.tenv).split("struct GenPayoff")[1]
    # too long to write out: the generic function serves that environment
    assert pay3.source(c3.tenv) == pay3.source()
