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


def _cl_inputs():
    from test_host_cl import CONTRACTS, to_cl
    from test_oracle_cl import rand_contract
    texts = [" ".join(t.split()) for t, _ in CONTRACTS.values()]
    for seed in range(150):
        texts.append(to_cl(rand_contract(np.random.default_rng(100 + seed), 5)))
    g = np.random.default_rng(11)
    mutated = []
    for t in texts:
        for _ in range(4):
            k = int(g.integers(0, len(t)))
            op = g.integers(0, 5)
            if op == 0:
                mutated.append(t[:k])                                    # truncation
            elif op == 1:
                mutated.append(t[:k] + ")" + t[k:])                     # stray paren
            elif op == 2:
                mutated.append(t[:k] + t[k + 1:])                       # dropped character
            elif op == 3:
                mutated.append(t[:k] + " obs(S, " + t[k:])              # junk form
            else:
                mutated.append(t[:k] + " 99999999999999999999 " + t[k:])  # out-of-range numeral
    deep = ["scale(1.0, " * 5000 + "zero" + ")" * 5000,                  # contracts beyond the nesting limit
            "scale(" + "-" * 100000 + "1.0, zero)",                       # unary chain
            "scale(" + "(" * 100000 + "1.0" + ")" * 100000 + ", zero)",   # parentheses
            "translate(2147483647, " * 900 + "zero" + ")" * 900,          # large day sums (valid text)
            "translate(99999999999999999999, zero)", "scale(obs(S, 99999999999), zero)",
            "scale(obs(S, -2147483647), transfer(X, Y))", "scale(1e400, zero)", "all[" * 3000 + "zero",
            "", "(", "zero)", "ifWithin(", "translate(T,"]
    return texts, mutated + deep


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the HIP headers not available")
def test_contract_front_end_under_sanitizers(tmp_path):
    """The contract-language reader and compiler (and the payoff loader on
    its output), built with AddressSanitizer and UndefinedBehaviorSanitizer
    (g++, host code only), on the workload contracts, random contracts, their
    mutations, nesting far beyond the limit and out-of-range numerals: every
    valid text compiles and loads, nothing crashes, leaks or overflows."""
    exe = tmp_path / "cl_fuzz"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
           "-I" + os.path.join(os.path.dirname(HERE), "include"), os.path.join(HERE, "cl_fuzz.cpp"),
           os.path.join(CSRC, "cl.cpp"), os.path.join(CSRC, "ilc.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    valid, other = _cl_inputs()
    inp = "\n".join(valid + other) + "\n"
    r = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stderr[-3000:]
    rows = [tuple(int(v) for v in line.split()) for line in r.stdout.splitlines()]
    assert len(rows) == len(valid) + len(other)
    assert all(st == 0 and ld == 0 for st, ld in rows[:len(valid)]), rows[:len(valid)]
    assert sum(1 for st, _ in rows[len(valid):] if st != 0) > len(other) // 2   # malformed texts are refused
    assert rows[len(valid) + len(other) - 14][0] != 0 and rows[len(valid) + len(other) - 13][0] != 0
