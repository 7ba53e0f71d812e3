"""Builds libpmc.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpmc.so")

SOURCES = ["ilc.cpp", "api.cpp", "codegen.cpp", "risk.cpp", "mc_kernels.hip", "mlp_kernels.hip", "mlp_api.cpp",
           "probe.hip", "cl.cpp"]
# Device engine sources embedded as text for run-time compilation of payoffs.
ENGINE_TEXT = ["pmc_device.h", "mc_engine.h"]
# Packed-FP32 instructions are disabled for every HIP translation unit.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include", "-I" + BUILD]


def _engine_inc():
    """Writes _build/engine_src.inc: the device engine as one string literal
    (local includes and include guards dropped; hipRTC provides the HIP
    runtime declarations)."""
    parts = []
    for name in ENGINE_TEXT:
        lines = open(os.path.join(CSRC, name)).read().splitlines()
        parts.append("\n".join(l for l in lines if not l.startswith('#include "') and l.strip() != "#pragma once"))
    text = "\n".join(parts)
    assert ')PMCSRC"' not in text
    out = 'static const char kEngineSource[] = R"PMCSRC(\n' + text + '\n)PMCSRC";\n'
    path = os.path.join(BUILD, "engine_src.inc")
    if not os.path.exists(path) or open(path).read() != out:
        open(path, "w").write(out)


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{out}")
    return obj, out


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    _engine_inc()
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    objs = []
    for obj, out in results:
        objs.append(obj)
        if verbose and out.strip():
            print(out)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + \
          ["-L/opt/rocm/lib", "-lrocrand", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
