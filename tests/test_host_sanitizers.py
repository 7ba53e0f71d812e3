"""The host-side loader built with AddressSanitizer and UndefinedBehavior-
Sanitizer (g++, host code only) survives valid, random and mutated IL texts
(CPU only)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2108_03076_amd", "csrc")


def _inputs():
    from oracle import cl
    from test_oracle_cl import rand_contract
    texts = [W.EUROPEAN_CALL, W.DOWN_AND_OUT_CALL, W.WORST_OF_AUTOCALL]
    for seed in range(150):
        texts.append(cl.to_text(cl.compile_contract(rand_contract(np.random.default_rng(seed), 5))))
    g = np.random.default_rng(7)
    mutated = []
    for t in texts:
        t = " ".join(t.split())
        for _ in range(4):
            k = int(g.integers(0, len(t)))
            op = g.integers(0, 4)
            if op == 0:
                mutated.append(t[:k])                             # truncation
            elif op == 1:
                mutated.append(t[:k] + ")" + t[k:])              # stray paren
            elif op == 2:
                mutated.append(t[:k] + t[k + 1:])                # dropped character
            else:
                mutated.append(t[:k] + " (tvar zz) " + t[k:])     # junk form
    deep = "(real 1.0)"
    for _ in range(3000):
        deep = f"(neg {deep})"
    return [" ".join(t.split()) for t in texts] + mutated + [deep, "", "(", ")", "(((((", "(real 1e400)",
                                                                "(model S (int -99999999999999999999))"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_loader_under_sanitizers(tmp_path):
    exe = tmp_path / "ilc_fuzz"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I" + CSRC, "-I" + os.path.join(os.path.dirname(HERE), "include"),
           os.path.join(HERE, "ilc_fuzz.cpp"), os.path.join(CSRC, "ilc.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    inp = "\n".join(_inputs()) + "\n"
    r = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stderr[-3000:]
    codes = [int(x) for x in r.stdout.split()]
    assert len(codes) == len(_inputs())
    assert codes[:153].count(0) == 153          # every valid text loads
    assert any(c != 0 for c in codes[153:])     # mutations are rejected, not crashed on
